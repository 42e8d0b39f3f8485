// RandFunmDiag gather (Section 3.3, Eq. rand_funm_formula_diag): one
// workgroup per start row k.
//
//  1. Q_k is built in LDS from the row's visit records: an open-addressing
//     hash table (keys int32, values FP64, linear probing, LDS atomics)
//     plus a one-bit-per-bucket filter that answers most misses with a
//     single LDS read.
//  2. For every requested row i adjacent to k, the column C_i (= row i, A is
//     symmetric) is streamed from memory and probed against Q_k:
//         dacc[i] += s a_ki * s <Q_k, C_i> / N      (FP64 atomic add)
//     Rows up to kBigRow entries go one per wavefront; longer rows are
//     streamed by the whole workgroup.
//  When the row's visits cannot fit the table at once, the walks are taken
//  in passes (Q_k is linear in the walks) and the gather repeats per pass.
#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

constexpr int kGatherThreads = 1024;
constexpr int kWaves = kGatherThreads / 64;
constexpr uint32_t kFilterLog2 = 16; // 65536 filter bits = 8 KiB
constexpr uint32_t kFilterWords = (1u << kFilterLog2) / 32;
constexpr uint32_t kBigRow = 2048;
constexpr uint32_t kBigQueue = 1024; // long rows queued per start row and pass
constexpr int32_t kEmpty = -1;

__device__ __forceinline__ uint32_t slot_of(int32_t key, uint32_t cap) {
    const uint32_t h = static_cast<uint32_t>(key) * 0x9E3779B1u;
    return __umulhi(h, cap);
}

__device__ __forceinline__ uint32_t filter_bit(int32_t key) {
    return (static_cast<uint32_t>(key) * 0x85EBCA77u) >> (32 - kFilterLog2);
}

struct Table {
    int32_t *keys;
    double *vals;
    uint32_t *filter;
    uint32_t cap;

    __device__ void insert(int32_t key, double x) {
        const uint32_t fb = filter_bit(key);
        atomicOr(&filter[fb >> 5], 1u << (fb & 31));
        uint32_t s = slot_of(key, cap);
        while (true) {
            const int32_t prev = atomicCAS(&keys[s], kEmpty, key);
            if (prev == kEmpty || prev == key) {
                atomicAdd(&vals[s], x);
                return;
            }
            s = (s + 1 == cap) ? 0 : s + 1;
        }
    }

    __device__ double lookup(int32_t key) const {
        const uint32_t fb = filter_bit(key);
        if (!((filter[fb >> 5] >> (fb & 31)) & 1u))
            return 0.0;
        uint32_t s = slot_of(key, cap);
        while (true) {
            const int32_t kv = keys[s];
            if (kv == key)
                return vals[s];
            if (kv == kEmpty)
                return 0.0;
            s = (s + 1 == cap) ? 0 : s + 1;
        }
    }
};

struct GatherArgs {
    const uint2 *node;
    const int32_t *col;
    const double *val;
    const int32_t *starts;
    int64_t n_start;
    int64_t N;
    int K;
    int64_t walks_per_pass;
    const int32_t *vstate;
    const double *vx;
    const uint8_t *in_set; // null: every row requested
    double scale;
    uint32_t cap;
    double *dacc;
    unsigned long long *probes;
};

template <bool WEIGHTED>
__device__ __forceinline__ double probe_row(const Table &tab, const GatherArgs &a, uint2 ri,
                                            uint32_t first, uint32_t stride) {
    double sum = 0.0;
    for (uint32_t e = first; e < ri.y; e += stride) {
        const int64_t idx = int64_t(ri.x) + e;
        const double qv = tab.lookup(a.col[idx]);
        sum += WEIGHTED ? a.val[idx] * qv : qv;
    }
    return sum;
}

template <bool WEIGHTED>
__global__ __launch_bounds__(kGatherThreads) void k_diag_gather(GatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double red[kWaves];
    __shared__ uint32_t big_queue[kBigQueue];
    __shared__ uint32_t big_count_s;
    uint32_t *big_count = &big_count_s;
    Table tab;
    tab.cap = a.cap;
    tab.vals = reinterpret_cast<double *>(smem);
    tab.keys = reinterpret_cast<int32_t *>(smem + sizeof(double) * a.cap);
    tab.filter = reinterpret_cast<uint32_t *>(smem + sizeof(double) * a.cap +
                                              sizeof(int32_t) * ((a.cap + 3) & ~3u));
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t span = int64_t(a.K - 1) * a.N;
    const double inv_n = 1.0 / static_cast<double>(a.N);
    unsigned long long probes = 0;

    for (int64_t kk = blockIdx.x; kk < a.n_start; kk += gridDim.x) {
        const int32_t k = a.starts[kk];
        const uint2 rk = a.node[k];
        const int32_t *st = a.vstate + kk * span;
        const double *xs = a.vx + kk * span;
        for (int64_t w0 = 0; w0 < a.N; w0 += a.walks_per_pass) {
            const int64_t nw = (a.N - w0 < a.walks_per_pass) ? (a.N - w0) : a.walks_per_pass;
            // (1) Q_k from walks [w0, w0 + nw).
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < a.cap; i += blockDim.x) {
                tab.keys[i] = kEmpty;
                tab.vals[i] = 0.0;
            }
            for (uint32_t i = threadIdx.x; i < kFilterWords; i += blockDim.x)
                tab.filter[i] = 0u;
            if (threadIdx.x == 0)
                *big_count = 0u;
            __syncthreads();
            const int64_t count = nw * (a.K - 1);
            if (nw == a.N) {
                for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
                    const int32_t s = st[i];
                    if (s >= 0)
                        tab.insert(s, xs[i]);
                }
            } else {
                for (int64_t i = threadIdx.x; i < count; i += blockDim.x) {
                    const int64_t t = i / nw;
                    const int64_t slot = t * a.N + w0 + (i - t * nw);
                    const int32_t s = st[slot];
                    if (s >= 0)
                        tab.insert(s, xs[slot]);
                }
            }
            __syncthreads();
            // (2a) requested neighbours with short rows: one wavefront each.
            //      Long rows are queued for (2b); a full queue makes the
            //      wavefront take the row itself.
            for (uint32_t p = wave; p < rk.y; p += kWaves) {
                const int64_t e = int64_t(rk.x) + p;
                const int32_t i = a.col[e];
                if (a.in_set && !a.in_set[i])
                    continue;
                const uint2 ri = a.node[i];
                if (ri.y > kBigRow) {
                    uint32_t pos = 0;
                    if (lane == 0)
                        pos = atomicAdd(big_count, 1u);
                    pos = __shfl(pos, 0, 64);
                    if (pos < kBigQueue) {
                        if (lane == 0)
                            big_queue[pos] = p;
                        continue;
                    }
                }
                const double sum = dev::wave_sum(probe_row<WEIGHTED>(tab, a, ri, lane, 64));
                probes += lane == 0 ? ri.y : 0;
                if (lane == 0) {
                    const double aki = WEIGHTED ? a.val[e] : 1.0;
                    atomicAdd(&a.dacc[i], (a.scale * aki) * (a.scale * sum) * inv_n);
                }
            }
            __syncthreads();
            // (2b) queued long rows: the whole workgroup streams each one.
            const uint32_t nbig = *big_count < kBigQueue ? *big_count : kBigQueue;
            for (uint32_t b = 0; b < nbig; ++b) {
                const uint32_t p = big_queue[b];
                const int64_t e = int64_t(rk.x) + p;
                const int32_t i = a.col[e];
                const uint2 ri = a.node[i];
                const double part = probe_row<WEIGHTED>(tab, a, ri, threadIdx.x, blockDim.x);
                const double sum = dev::block_sum(part, red);
                if (threadIdx.x == 0) {
                    probes += ri.y;
                    const double aki = WEIGHTED ? a.val[e] : 1.0;
                    atomicAdd(&a.dacc[i], (a.scale * aki) * (a.scale * sum) * inv_n);
                }
            }
        }
    }
    if (a.probes) {
        const unsigned long long total = dev::block_sum(probes, reinterpret_cast<unsigned long long *>(red));
        if (threadIdx.x == 0)
            atomicAdd(a.probes, total);
    }
}

} // namespace

// Table capacity and walks per pass for a row with N walks of K-1 visits.
void gather_plan(int64_t n, int64_t N, int K, uint32_t *cap, int64_t *walks_per_pass,
                 size_t *lds_bytes) {
    const size_t lds_max = 160 * 1024;
    const size_t fixed = sizeof(uint32_t) * kFilterWords + sizeof(double) * kWaves +
                         sizeof(uint32_t) * (kBigQueue + 1) + 256;
    const uint32_t cap_max = static_cast<uint32_t>(((lds_max - fixed) / 12) & ~63u);
    const int64_t visits = N * (K - 1);
    int64_t distinct = visits < n ? visits : n;
    int64_t wpp = N;
    // Load factor at most 0.8 in the worst case (every visit distinct).
    if (distinct * 5 > int64_t(cap_max) * 4) {
        wpp = (int64_t(cap_max) * 4 / 5) / (K - 1);
        if (wpp < 1)
            wpp = 1;
        if (n * 5 <= int64_t(cap_max) * 4)
            wpp = N; // few nodes: the table holds them all whatever the walk count
        const int64_t v = wpp * (K - 1);
        distinct = v < n ? v : n;
    }
    uint32_t c = static_cast<uint32_t>((distinct * 5 + 3) / 4 + 1);
    c = (c + 63) & ~63u;
    if (c < 64)
        c = 64;
    if (c > cap_max)
        c = cap_max;
    *cap = c;
    *walks_per_pass = wpp;
    *lds_bytes = sizeof(double) * c + sizeof(int32_t) * ((c + 3) & ~3u) + sizeof(uint32_t) * kFilterWords;
}

Status diag_gather(const mcmf_graph *g, const int32_t *starts, int64_t n_start, const WalkParams &p,
                   const int32_t *state, const double *x, const uint8_t *in_set, double *dacc,
                   unsigned long long *probes, hipStream_t s) {
    if (n_start <= 0 || p.K < 2)
        return {};
    GatherArgs a = {};
    a.node = g->node;
    a.col = g->col;
    a.val = g->val;
    a.starts = starts;
    a.n_start = n_start;
    a.N = p.n_walks;
    a.K = p.K;
    a.vstate = state;
    a.vx = x;
    a.in_set = in_set;
    a.scale = p.scale;
    a.dacc = dacc;
    a.probes = probes;
    size_t lds = 0;
    gather_plan(g->n, p.n_walks, p.K, &a.cap, &a.walks_per_pass, &lds);
    const int64_t cap_blocks = int64_t(1) << 20;
    const dim3 grid(static_cast<uint32_t>(n_start < cap_blocks ? n_start : cap_blocks));
    if (g->weighted) {
        MCMF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_diag_gather<true>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(k_diag_gather<true>, grid, dim3(kGatherThreads), lds, s, a);
    } else {
        MCMF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&k_diag_gather<false>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(k_diag_gather<false>, grid, dim3(kGatherThreads), lds, s, a);
    }
    MCMF_HIP(hipGetLastError());
    return {};
}

} // namespace mcmf
