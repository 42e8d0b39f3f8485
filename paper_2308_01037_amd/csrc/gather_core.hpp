// Device-side core of the diagonal gather (Section 3.3, Eq.
// rand_funm_formula_diag) for one start row k, shared by the single-request
// and the batched gather kernels.
//
//  1. Q_k is built in LDS from the row's visit records: open addressing over
//     8-slot buckets (keys int32, values FP64, LDS atomics on insert) and a
//     blocked three-bit filter that rejects most absent keys with one LDS
//     read.  A lookup reads a whole bucket (two 16-byte reads) per step.
//  2. The columns C_i (= row i, A is symmetric) of the requested neighbours i
//     of k, 256 neighbours at a time, are cut into chunks of kChunk entries.
//     A group of 16 lanes takes a contiguous range of chunks (8 entries per
//     lane, coalesced, all loads in flight together), probes Q_k for each
//     entry, sums over the group and adds the sum into the neighbour's LDS
//     total; after the batch each neighbour's total goes out with one FP64
//     atomic:   dacc[i] += s a_ki * s <Q_k, C_i> / N.
//  3. Hub rows (unweighted graphs): for a neighbour h of k among the graph's
//     active hubs (its highest-degree rows), <Q_k, C_h> is summed by the walk
//     kernel instead (it sees each state's hub mask in the edge record it
//     loads anyway); every item leaves those neighbours out of step 2.
//  4. Small items (one batch of neighbours whose column entries number at
//     most half the visits): the table first takes those entries as keys,
//     then each visit is added to its key if present.  Q_k restricted to the
//     entries the probes ask for gives the same inner products with one
//     lookup per visit instead of one insert.
//  When the row's visits cannot fit the table at once, the walks are taken
//  in passes (Q_k is linear in the walks) and the gather repeats per pass.
#pragma once

#include <mutex>
#include <set>
#include <utility>

#include "device.hpp"
#include "ops.hpp"
#include "plan.hpp"

namespace mcmf {
namespace gather {

constexpr int kGatherThreads = 1024;
constexpr int kWaves = kGatherThreads / 64;
constexpr uint32_t kFilterLog2Words = 11; // 2048 words = 8 KiB
constexpr uint32_t kFilterWords = 1u << kFilterLog2Words;
constexpr int kBatch = 256;                // neighbours per batch
constexpr int kGroup = 16;                 // lanes per chunk
constexpr int kPerLane = 8;                // entries per lane per chunk
constexpr int kChunk = kGroup * kPerLane;  // entries per chunk
constexpr int kGroups = kGatherThreads / kGroup;
constexpr int kSlots = 8;                  // slots per bucket
constexpr int kVisits = 4;                 // visit records per thread in flight (table build)
constexpr int32_t kEmpty = -1;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    // Multiply-xorshift integer hash (the finaliser of MurmurHash3).
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

struct Table {
    int32_t *keys; // nb buckets x kSlots slots, 32-byte aligned
    double *vals;
    uint32_t *filter;
    uint32_t nb;

    // Empties the first cap slots and the filter (all threads of the block,
    // between barriers).
    __device__ void clear(uint32_t cap) const {
        for (uint32_t i = threadIdx.x; i < cap; i += blockDim.x) {
            keys[i] = kEmpty;
            vals[i] = 0.0;
        }
        for (uint32_t i = threadIdx.x; i < kFilterWords; i += blockDim.x)
            filter[i] = 0u;
    }

    // Multiplicative hashing: node ids of the graphs here carry no structure
    // that a multiply-shift hash would keep.
    __device__ __forceinline__ uint32_t bucket_of(int32_t key) const {
        return __umulhi(static_cast<uint32_t>(key) * 0x85EBCA77u, nb);
    }
    __device__ __forceinline__ static uint32_t fhash(int32_t key) {
        return static_cast<uint32_t>(key) * 0x9E3779B1u;
    }
    // Top bits pick the filter word, three 5-bit fields below them the bits.
    __device__ __forceinline__ static uint32_t filter_word(uint32_t h) {
        return h >> (32 - kFilterLog2Words);
    }
    __device__ __forceinline__ static uint32_t filter_mask(uint32_t h) {
        return (1u << ((h >> 6) & 31)) | (1u << ((h >> 11) & 31)) | (1u << (h & 31));
    }

    // Slot of key in a bucket read as (lo, hi), or -1.
    __device__ __forceinline__ static int slot_in(const int4 &lo, const int4 &hi, int32_t key) {
        int j = -1;
        j = (lo.x == key) ? 0 : j;
        j = (lo.y == key) ? 1 : j;
        j = (lo.z == key) ? 2 : j;
        j = (lo.w == key) ? 3 : j;
        j = (hi.x == key) ? 4 : j;
        j = (hi.y == key) ? 5 : j;
        j = (hi.z == key) ? 6 : j;
        j = (hi.w == key) ? 7 : j;
        return j;
    }

    // Adds x to key's value, claiming a slot for a new key.  Each pass reads
    // the bucket once: a present key gets the add; otherwise the first empty
    // slot is claimed with one compare-and-swap (slots fill in order, so no
    // key sits behind an empty slot).  A lost claim means another key took
    // that slot, so the bucket is read again; a full bucket passes the probe
    // on.  Every lost claim fills a slot, which bounds the passes.  Returns
    // false only if every bucket is full (the plan rules that out).
    // Slot of key, claimed for it if the key is new, or -1 if every bucket is
    // full (the plan rules that out).
    __device__ int claim_slot(int32_t key) const {
        const uint32_t h = fhash(key);
        atomicOr(&filter[filter_word(h)], filter_mask(h));
        uint32_t b = bucket_of(key);
        const uint32_t max_passes = (kSlots + 1) * nb;
        for (uint32_t pass = 0; pass < max_passes; ++pass) {
            const int4 lo = *reinterpret_cast<const int4 *>(keys + kSlots * b);
            const int4 hi = *reinterpret_cast<const int4 *>(keys + kSlots * b + 4);
            const int j = slot_in(lo, hi, key);
            if (j >= 0)
                return static_cast<int>(kSlots * b) + j;
            const int used = (lo.x != kEmpty) + (lo.y != kEmpty) + (lo.z != kEmpty) +
                             (lo.w != kEmpty) + (hi.x != kEmpty) + (hi.y != kEmpty) +
                             (hi.z != kEmpty) + (hi.w != kEmpty);
            if (used == kSlots) {
                b = (b + 1 == nb) ? 0 : b + 1;
                continue;
            }
            const uint32_t s = kSlots * b + used;
            const int32_t prev = atomicCAS(&keys[s], kEmpty, key);
            if (prev == kEmpty || prev == key)
                return static_cast<int>(s);
        }
        return -1;
    }

    __device__ bool insert(int32_t key, double x) const {
        const int s = claim_slot(key);
        if (s < 0)
            return false;
        atomicAdd(&vals[s], x);
        return true;
    }

    // Slot of key, or -1 when it is absent (no insert may run meanwhile).
    __device__ int locate(int32_t key) const {
        const uint32_t h = fhash(key);
        const uint32_t m = filter_mask(h);
        if ((filter[filter_word(h)] & m) != m)
            return -1;
        uint32_t b = bucket_of(key);
        for (uint32_t tries = 0; tries < nb; ++tries) {
            const int4 lo = *reinterpret_cast<const int4 *>(keys + kSlots * b);
            const int4 hi = *reinterpret_cast<const int4 *>(keys + kSlots * b + 4);
            const int j = slot_in(lo, hi, key);
            if (j >= 0)
                return static_cast<int>(kSlots * b) + j;
            if (hi.w == kEmpty)
                return -1; // slots fill in order: the key would be here
            b = (b + 1 == nb) ? 0 : b + 1;
        }
        return -1;
    }

    // Value of key in bucket b, or: 0 with *more = false when the key is absent
    // (an empty slot ends the probe sequence), *more = true when the bucket is
    // full without it (continue with the next bucket).
    __device__ __forceinline__ double probe_bucket(int32_t key, uint32_t b, bool *more) const {
        const int4 lo = *reinterpret_cast<const int4 *>(keys + kSlots * b);
        const int4 hi = *reinterpret_cast<const int4 *>(keys + kSlots * b + 4);
        const int j = slot_in(lo, hi, key);
        *more = false;
        if (j >= 0)
            return vals[kSlots * b + j];
        *more = hi.w != kEmpty; // slots fill in order: the last one is the test
        return 0.0;
    }

    // acc + sum_u w[u] Q[key[u]] (w[u] = 1 unweighted) over N keys, looked up
    // stage by stage so that their LDS reads overlap: all filter words, then
    // the home buckets and values in two halves (to bound register use), then
    // the rare keys that need further buckets.  key < 0 means "no key".
    template <int N, bool WEIGHTED>
    __device__ __forceinline__ double lookup_sum(const int32_t (&key)[N], const double (&w)[N],
                                                 double acc) const {
        static_assert(N % 2 == 0, "N must be even");
        constexpr int H = N / 2;
        uint32_t fw[N], m[N];
#pragma unroll
        for (int u = 0; u < N; ++u) {
            // Every lane reads a filter word (any word serves for "no key").
            const uint32_t h = fhash(key[u]);
            m[u] = filter_mask(h);
            fw[u] = filter[filter_word(h)];
        }
        uint32_t pending = 0;
#pragma unroll
        for (int half = 0; half < 2; ++half) {
            // Every lane issues its reads; lanes without a candidate read bucket
            // 0, one address the LDS serves as a broadcast.
            bool cand[H];
            uint32_t b[H];
            int4 lo[H], hi[H];
#pragma unroll
            for (int v = 0; v < H; ++v) {
                const int u = half * H + v;
                cand[v] = key[u] >= 0 && (fw[u] & m[u]) == m[u];
                const uint32_t home = bucket_of(key[u]);
                b[v] = cand[v] ? home : 0u;
                lo[v] = *reinterpret_cast<const int4 *>(keys + kSlots * b[v]);
                hi[v] = *reinterpret_cast<const int4 *>(keys + kSlots * b[v] + 4);
            }
            int slot[H];
#pragma unroll
            for (int v = 0; v < H; ++v) {
                const int u = half * H + v;
                int j = slot_in(lo[v], hi[v], key[u]);
                j = cand[v] ? j : -1;
                // Slots fill in order, so a full bucket ends with a used last slot.
                pending |= (cand[v] && j < 0 && hi[v].w != kEmpty) ? (1u << u) : 0u;
                slot[v] = j;
            }
            double got[H];
#pragma unroll
            for (int v = 0; v < H; ++v)
                got[v] = vals[slot[v] >= 0 ? kSlots * b[v] + slot[v] : 0u];
#pragma unroll
            for (int v = 0; v < H; ++v) {
                const double q = slot[v] >= 0 ? got[v] : 0.0;
                acc += WEIGHTED ? w[half * H + v] * q : q;
            }
        }
        while (pending) {
            const int u = __ffs(pending) - 1;
            pending &= pending - 1;
            int32_t kx = key[0];
#pragma unroll
            for (int v = 1; v < N; ++v)
                kx = (v == u) ? key[v] : kx;
            uint32_t bx = bucket_of(kx);
            double r = 0.0;
            bool more = true;
            for (uint32_t tries = 1; more && tries < nb; ++tries) {
                bx = (bx + 1 == nb) ? 0 : bx + 1;
                r = probe_bucket(kx, bx, &more);
            }
            if constexpr (WEIGHTED) {
                double wx = w[0];
#pragma unroll
                for (int v = 1; v < N; ++v)
                    wx = (v == u) ? w[v] : wx;
                acc += wx * r;
            } else {
                acc += r;
            }
        }
        return acc;
    }
};

// Per-batch neighbour metadata in LDS.
struct Batch {
    uint32_t prefix[kBatch + 1]; // first chunk of each neighbour's column
    uint32_t start[kBatch];      // first entry of the column in col[]
    uint32_t len[kBatch];        // column length
    int32_t row[kBatch];         // neighbour i (-1: not requested)
    double aki[kBatch];          // s * a_ki
    double sum[kBatch];          // <Q_k, C_i> partial sums
};

// LDS views shared by every row a workgroup processes.
struct Shared {
    Table tab;
    Batch *bt;
    uint32_t *scan_scratch; // one word per wavefront
    unsigned long long *red; // one word per wavefront
};

// One start row's gather job.
struct RowJob {
    int32_t k;
    uint2 rk;               // record of row k
    uint32_t p_begin, p_end; // neighbours [p_begin, p_end) of row k (positions in its row)
    const int32_t *st;      // visit states of row k, t-major (t * N + w)
    int64_t N;              // walks of row k
    int K;
    int64_t walks_per_pass;
    const uint2 *node;
    const int32_t *col;
    const double *val;
    const uint8_t *in_set;  // null: every row requested
    double scale;
    double *dacc;
    unsigned long long *overflow;
    const uint8_t *hub_of;   // per node: its hub index, or kNoHub
    uint32_t hub_act;        // hubs summed by the walks, not probed here (0: none)
    const uint16_t *whub_of; // per node: its wide hub index, or kNoWideHub
    int32_t whub_act;        // wide hubs [0, whub_act) summed by the walks (0: none)
};

// Runs the job with all threads of the workgroup (kGatherThreads).
template <bool WEIGHTED, class VT>
__device__ void gather_row(const Shared &sh, const RowJob &j, const VT *__restrict__ xs,
                           unsigned long long &probes) {
    const Table &tab = sh.tab;
    Batch &bt = *sh.bt;
    uint32_t *scan_scratch = sh.scan_scratch;
    const uint32_t cap = kSlots * tab.nb;
    const double inv_n = 1.0 / static_cast<double>(j.N);
    const int32_t k = j.k;
    const uint2 rk = j.rk;
    const int32_t *st = j.st;
    const int group = threadIdx.x / kGroup;
    const int gl = threadIdx.x % kGroup;

    // Neighbours [p0, p0 + m) of k into bt; returns the number of column
    // chunks (kChunk entries each) of those that are requested and probed.
    // The first batch of a job needs no barrier of its own: the caller's
    // barrier before the job, or the one after the table is cleared, already
    // separates it from the last reads of bt and of scan_scratch.
    auto setup_batch = [&](uint32_t p0, uint32_t m) -> uint32_t {
        if (p0 != j.p_begin)
            __syncthreads(); // previous batch flushed
        uint32_t nchunks = 0;
        if (threadIdx.x < kBatch) {
            const int t = threadIdx.x;
            bt.sum[t] = 0.0;
            bt.row[t] = -1;
            bt.len[t] = 0;
            if (uint32_t(t) < m) {
                const int64_t e = int64_t(rk.x) + p0 + t;
                const int32_t i = j.col[e];
                bool take = !j.in_set || j.in_set[i];
                if constexpr (!WEIGHTED) {
                    // Active hubs are summed by the walks instead.
                    if (take && j.hub_act != 0u) {
                        const uint32_t hx = j.hub_of[i];
                        take = hx == kNoHub || ((j.hub_act >> hx) & 1u) == 0u;
                    }
                    if (take && j.whub_act > 0)
                        take = static_cast<int32_t>(j.whub_of[i]) >= j.whub_act;
                }
                if (take) {
                    const uint2 ri = j.node[i];
                    nchunks = (ri.y + kChunk - 1) / kChunk;
                    bt.start[t] = ri.x;
                    bt.len[t] = ri.y;
                    bt.row[t] = i;
                    bt.aki[t] = j.scale * (WEIGHTED ? j.val[e] : 1.0);
                }
            }
        }
        uint32_t total = 0;
        const uint32_t before = dev::block_exclusive_scan(nchunks, scan_scratch, &total, true);
        if (threadIdx.x < kBatch)
            bt.prefix[threadIdx.x] = before;
        if (threadIdx.x == 0)
            bt.prefix[kBatch] = total;
        __syncthreads();
        return total;
    };
    // First neighbour (in bt) whose chunks reach chunk c.
    auto owner = [&](uint32_t c) -> int {
        int r = 0, hi = kBatch;
        while (hi - r > 1) {
            const int mid = (r + hi) >> 1;
            if (bt.prefix[mid] <= c)
                r = mid;
            else
                hi = mid;
        }
        return r;
    };

    for (int64_t w0 = 0; w0 < j.N; w0 += j.walks_per_pass) {
        const int64_t nw = (j.N - w0 < j.walks_per_pass) ? (j.N - w0) : j.walks_per_pass;
        const int64_t count = nw * (j.K - 1);
        // An item of one neighbour batch whose columns hold fewer entries than
        // half the visits: the table takes those entries as keys and the
        // visits are added to the keys present (Q_k restricted to the entries
        // the probes will ask for), instead of every visit being inserted.
        const bool single = nw == j.N && j.p_end - j.p_begin <= uint32_t(kBatch);
        uint32_t total0 = 0;
        bool restricted = false;
        if (single) {
            // The last probe of the previous job came before a barrier; the
            // batch setup's barriers order this clear before the inserts.
            tab.clear(cap);
            total0 = setup_batch(j.p_begin, j.p_end - j.p_begin);
            // Nothing to probe (every neighbour unrequested or summed by the
            // walk): no table either.
            if (total0 == 0)
                continue;
            // total0 * kChunk bounds the batch's column entries from above.
            restricted = uint64_t(total0) * kChunk * kRestrictNum <= static_cast<uint64_t>(count) * kRestrictDen;
        }
        if (!single) {
            // The last probe of the previous pass or job came before a barrier.
            tab.clear(cap);
            __syncthreads();
        }
        if (restricted) {
            // (1') the column entries of the batch as keys.
            const uint32_t per = (total0 + kGroups - 1) / kGroups;
            const uint32_t c_begin = group * per;
            const uint32_t c_end = (c_begin + per < total0) ? c_begin + per : total0;
            if (c_begin < c_end) {
                int r = owner(c_begin);
                for (uint32_t c = c_begin; c < c_end; ++c) {
                    while (c >= bt.prefix[r + 1])
                        ++r;
                    const uint32_t off0 = (c - bt.prefix[r]) * kChunk;
                    const uint32_t len = bt.len[r];
                    const int64_t base = int64_t(bt.start[r]);
#pragma unroll
                    for (int u = 0; u < kPerLane; ++u) {
                        const uint32_t off = off0 + gl + u * kGroup;
                        if (off < len && tab.claim_slot(j.col[base + off]) < 0)
                            atomicAdd(j.overflow, 1ull);
                    }
                }
            }
            __syncthreads();
            // (2') every visit added to its key when the key is present.
            // Step 0 of every walk sits at k: its visits are summed per
            // wavefront and added once per wavefront, after the others, so
            // that their loads overlap the loop's and no barrier is needed.
            double x0 = 0.0;
            for (int64_t i = threadIdx.x; i < nw; i += blockDim.x)
                x0 += st[i] >= 0 ? static_cast<double>(xs[i]) : 0.0;
            for (int64_t i0 = nw + threadIdx.x; i0 < count; i0 += kVisits * int64_t(blockDim.x)) {
                int32_t sv[kVisits];
                double xv[kVisits];
#pragma unroll
                for (int u = 0; u < kVisits; ++u) {
                    const int64_t i = i0 + int64_t(u) * blockDim.x;
                    sv[u] = i < count ? st[i] : -1;
                    xv[u] = i < count ? static_cast<double>(xs[i]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kVisits; ++u) {
                    const int sl = sv[u] >= 0 ? tab.locate(sv[u]) : -1;
                    if (sl >= 0)
                        atomicAdd(&tab.vals[sl], xv[u]);
                }
            }
            x0 = dev::wave_sum(x0);
            if ((threadIdx.x & 63) == 0 && x0 != 0.0) {
                const int sk = tab.locate(k);
                if (sk >= 0)
                    atomicAdd(&tab.vals[sk], x0);
            }
        } else if (nw == j.N) {
            // (1) Q_k from all walks.  Step 0 of every walk sits at k: those
            // visits are summed per wavefront and inserted once per
            // wavefront, after the others, instead of N colliding atomic
            // updates of one slot (and with no barrier of their own).
            double x0 = 0.0;
            for (int64_t i = threadIdx.x; i < nw; i += blockDim.x)
                x0 += st[i] >= 0 ? static_cast<double>(xs[i]) : 0.0;
            // kVisits records per thread: their loads are issued together
            // before the inserts.
            for (int64_t i0 = nw + threadIdx.x; i0 < count; i0 += kVisits * int64_t(blockDim.x)) {
                int32_t sv[kVisits];
                double xv[kVisits];
#pragma unroll
                for (int u = 0; u < kVisits; ++u) {
                    const int64_t i = i0 + int64_t(u) * blockDim.x;
                    sv[u] = i < count ? st[i] : -1;
                    xv[u] = i < count ? static_cast<double>(xs[i]) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kVisits; ++u)
                    if (sv[u] >= 0 && !tab.insert(sv[u], xv[u]))
                        atomicAdd(j.overflow, 1ull);
            }
            x0 = dev::wave_sum(x0);
            if ((threadIdx.x & 63) == 0 && x0 != 0.0 && !tab.insert(k, x0))
                atomicAdd(j.overflow, 1ull);
        } else {
            // (1) Q_k from walks [w0, w0 + nw).
            for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
                const int64_t t = i / nw;
                const int64_t slot = t * j.N + w0 + (i - t * nw);
                const int32_t s = st[slot];
                if (s >= 0 && !tab.insert(s, static_cast<double>(xs[slot])))
                    atomicAdd(j.overflow, 1ull);
            }
        }
        // (2) columns of the requested neighbours, kBatch neighbours at a time.
        for (uint32_t p0 = j.p_begin; p0 < j.p_end; p0 += kBatch) {
            const uint32_t m = (j.p_end - p0 < uint32_t(kBatch)) ? j.p_end - p0 : uint32_t(kBatch);
            uint32_t total;
            if (single) {
                __syncthreads(); // table complete (the batch is already in bt)
                total = total0;
            } else {
                total = setup_batch(p0, m);
            }
            // Group g takes the contiguous chunk range [g*per, (g+1)*per) and
            // walks the neighbours forward, so the owner is searched once.
            const uint32_t per = (total + kGroups - 1) / kGroups;
            const uint32_t c_begin = group * per;
            const uint32_t c_end = (c_begin + per < total) ? c_begin + per : total;
            if (c_begin < c_end) {
                int r = owner(c_begin);
                uint32_t next = bt.prefix[r + 1];
                uint32_t len = bt.len[r];
                int64_t base = int64_t(bt.start[r]);
                uint32_t first_chunk = bt.prefix[r];
                double acc = 0.0;
                for (uint32_t c = c_begin; c < c_end; ++c) {
                    if (c >= next) {
                        // Row change: flush the finished neighbour's partial sum.
                        const double g = dev::group_sum<kGroup>(acc);
                        if (gl == 0 && g != 0.0)
                            atomicAdd(&bt.sum[r], g);
                        acc = 0.0;
                        do {
                            ++r;
                            next = bt.prefix[r + 1];
                        } while (c >= next);
                        len = bt.len[r];
                        base = int64_t(bt.start[r]);
                        first_chunk = bt.prefix[r];
                    }
                    const uint32_t off0 = (c - first_chunk) * kChunk;
                    const uint32_t first = off0 + gl;
                    int32_t key[kPerLane];
                    double wv[kPerLane];
                    if (off0 + kChunk <= len) {
#pragma unroll
                        for (int u = 0; u < kPerLane; ++u) {
                            key[u] = j.col[base + first + u * kGroup];
                            wv[u] = WEIGHTED ? j.val[base + first + u * kGroup] : 1.0;
                        }
                        probes += gl == 0 ? kChunk : 0;
                    } else {
#pragma unroll
                        for (int u = 0; u < kPerLane; ++u) {
                            const uint32_t off = first + u * kGroup;
                            key[u] = off < len ? j.col[base + off] : -1;
                            wv[u] = (WEIGHTED && off < len) ? j.val[base + off] : 1.0;
                        }
                        probes += gl == 0 ? len - off0 : 0;
                    }
                    acc = tab.lookup_sum<kPerLane, WEIGHTED>(key, wv, acc);
                }
                const double g = dev::group_sum<kGroup>(acc);
                if (gl == 0 && g != 0.0)
                    atomicAdd(&bt.sum[r], g);
            }
            __syncthreads();
            if (threadIdx.x < m && bt.row[threadIdx.x] >= 0) {
                const int t = threadIdx.x;
                atomicAdd(&j.dacc[bt.row[t]], bt.aki[t] * (j.scale * bt.sum[t]) * inv_n);
            }
        }
    }
}

// Work items.  A start row with d neighbours is cut into ceil(d / item)
// items of at most `item` neighbours each (the graph's tuning); every item
// builds Q_k itself, so the items of a high-degree row run on many
// workgroups at once.  item_off[kk] = first item of start row kk (exclusive
// prefix sums).
__device__ __forceinline__ uint32_t items_of(uint32_t deg, uint32_t item) {
    return (deg + item - 1) / item;
}

// Start row kk in [lo, hi) with off[kk] <= item < off[kk + 1].
__device__ __forceinline__ int64_t row_of_item(const int64_t *__restrict__ off, int64_t lo,
                                               int64_t hi, int64_t item) {
    while (hi - lo > 1) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if (off[mid] <= item)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// Next work item of the workgroup from a queue counter (one atomic per item,
// broadcast through LDS).
__device__ __forceinline__ int64_t next_item(unsigned long long *counter, int64_t *slot) {
    __syncthreads(); // every thread has read the previous item
    if (threadIdx.x == 0)
        *slot = static_cast<int64_t>(atomicAdd(counter, 1ull));
    __syncthreads();
    return *slot;
}

// LDS bytes of the table for a plan, and of the fixed per-workgroup arrays.
constexpr size_t kStaticLds = sizeof(Batch) + sizeof(uint32_t) * kWaves +
                              sizeof(unsigned long long) * kWaves + 512;

// Largest dynamic LDS (table + filter) a gather plan may ask for.
constexpr size_t kMaxTableLds = 160 * 1024 - kStaticLds;

// Raises a gather kernel's dynamic-LDS limit to kMaxTableLds, once per
// (kernel, device).  The limit is a property of the kernel shared by every
// host thread: setting it per call to that call's table size would let a
// concurrent call on another stream lower it under a launch of its own.
inline Status allow_table_lds(const void *fn) {
    static std::mutex mu;
    static std::set<std::pair<const void *, int>> done;
    int dev = 0;
    MCMF_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(mu);
    if (done.count({fn, dev}))
        return {};
    MCMF_HIP(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 static_cast<int>(kMaxTableLds)));
    done.insert({fn, dev});
    return {};
}

__device__ __forceinline__ Shared shared_views(unsigned char *smem, uint32_t nb, Batch *bt,
                                               uint32_t *scan, unsigned long long *red) {
    Shared sh;
    const uint32_t cap = kSlots * nb;
    sh.tab.nb = nb;
    sh.tab.vals = reinterpret_cast<double *>(smem);
    sh.tab.keys = reinterpret_cast<int32_t *>(smem + sizeof(double) * cap);
    sh.tab.filter = reinterpret_cast<uint32_t *>(smem + sizeof(double) * cap + sizeof(int32_t) * cap);
    sh.bt = bt;
    sh.scan_scratch = scan;
    sh.red = red;
    return sh;
}

} // namespace gather
} // namespace mcmf
