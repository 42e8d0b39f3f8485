// Batched execution (mcmf_batch): many diag / action requests as one unit of
// GPU work.
//
// Work items.  A walk task is 64 walks (one wavefront) of one start row of
// one request; the persistent walk kernel's wavefronts take tasks from the
// flattened task space of all requests, so requests with few walks per row
// or few rows do not leave the GPU idle.  Action tasks add their wavefront
// sum into q[k] (FP64 atomics); diagonal tasks write visit records.  The
// persistent gather workgroups then take items (up to 256 neighbours of one
// start row of one diagonal request) from a queue counter and run
// gather_core.hpp on each.  Diagonal visit records are produced and
// consumed in chunks bounded by a byte budget; all action tasks ride along in
// the first chunk's walk launch.
//
// Keyed walks: a task draws exactly the Philox counters its request's own
// mcmf_diag / mcmf_action call would draw, so results agree with those calls
// up to the order of floating-point additions.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <type_traits>
#include <utility>
#include <cstring>
#include <memory>
#include <vector>

#include "gather_core.hpp"
#include "walk_core.hpp"

namespace mcmf {

namespace {

constexpr int kWalkThreads = 256;

// Walk kernel variant of a request: FP32 weights, weighted graph, weight
// cutoff, path digest.
// kModeValue: an action request walking over its own value records (see
// walk_core.hpp, action_walk_value): unweighted graphs without a digest.
// kModeWide: a diagonal request with wide hub sums (diag_walk_wide), one
// start row per task: unweighted graphs whose layout is MCMF_SAMPLER_WIDE.
enum : int32_t { kModeFp32 = 1, kModeWeighted = 2, kModeCutoff = 4, kModeDigest = 8, kModeValue = 16,
                 kModeWide = 32 };
constexpr int kWalkModes = 64;

// Device descriptor of one request.
struct BReq {
    walk::GraphView g;
    walk::WalkArgs a;
    int32_t kind; // MCMF_REQ_*
    int32_t mode; // kMode* bits
    const int32_t *starts;
    const double *r;           // action: s A v
    double *q;                 // action: q per start row
    uint64_t *digest;          // optional
    unsigned long long *steps; // this request's step counter
    const uint8_t *in_set;     // diag subset (null: all rows)
    double *dacc;              // diag sums
    const int64_t *item_off;   // diag: gather work items of the start list
    int64_t wpp;               // walks per gather pass
    const uint4 *rec;          // action, value mode: this request's value records
    const uint8_t *hub_of;     // diag: hub index per node
    uint32_t hub_act;          // diag: hubs the walks sum (a.hub_act), left out of the probes
    uint32_t item;             // diag: neighbours per gather work item (the graph's tuning)
    // kModeWide: the graph's wide masks and hub rows, and the active prefix
    // of wide hubs the walks sum and the gather leaves out (0 otherwise).
    const uint32_t *wmask;
    const int32_t *whub_rows;
    const uint16_t *whub_of;
    int32_t whub_act;
};

// A run of one request's start rows inside a walk launch.  A task is one
// workgroup (256 threads): with N >= 128 walks per row, all N walks of one
// row (each thread loops over walks, as the single-request kernel does, so a
// row's walks share one CU and its caches); with N < 128, all N walks of
// rows_per_task = floor(256 / N) rows, one walk per thread.
struct WSeg {
    int32_t req;
    uint32_t rows_per_task; // 0: one row per task (N >= 128)
    int64_t kk0;            // first start-row index in the request's start list
    int64_t rows;           // start rows in the run
    int64_t task_base;      // first task of this run in the launch
    int64_t slot_base;      // diag: first visit slot of row kk0 in the chunk
    int64_t xoff;           // diag: byte offset of that slot's value
};

// A run of one request's start rows inside a gather launch.  item_base (the
// run's first work item in the launch) is filled in on the device; an extra
// entry after the last run holds the launch's item count.
struct GSeg {
    int32_t req;
    int64_t kk0;
    int64_t rows;
    int64_t item_base;
    int64_t slot_base;
    int64_t xoff;
};

constexpr int64_t kRowTaskWalks = 128; // N at or above which a task is one row
constexpr int64_t kHubMinWalks = 32;   // packed tasks hold at most 256/32 rows of hub sums
constexpr int kHubRows = kWalkThreads / kHubMinWalks;

template <class WT, bool WEIGHTED, bool CUTOFF, bool DIGEST, bool VALUE>
__device__ __forceinline__ void one_walk(const BReq &R, const WSeg &sg, int64_t rel, uint32_t k, uint2 rk,
                                         int64_t w, int32_t *vstate, unsigned char *vxb, double &acc,
                                         uint64_t &h, unsigned long long &ns, uint32_t hub_k = 0u,
                                         double *hsum = nullptr) {
    const int64_t N = R.a.N;
    if constexpr (VALUE) {
        // Only action requests carry the value mode.
        acc += walk::action_walk_value<WT, CUTOFF, false>(R.rec, R.a, k, rk, R.r[k], static_cast<uint32_t>(w),
                                                          &ns);
    } else if (R.kind == MCMF_REQ_ACTION) {
        acc += walk::action_walk<WT, WEIGHTED, DIGEST, CUTOFF>(R.g, R.r, R.a, k, rk, R.r[k],
                                                                static_cast<uint32_t>(w), &h, &ns);
    } else {
        const int64_t span = int64_t(R.a.K - 1) * N;
        WT *vx = reinterpret_cast<WT *>(vxb + sg.xoff) + rel * span;
        walk::diag_walk<WT, WEIGHTED, DIGEST, CUTOFF>(R.g, R.a, k, rk, static_cast<uint32_t>(w),
                                                       vstate + sg.slot_base + rel * span + w, vx + w, N,
                                                       &h, &ns, hub_k, hsum);
    }
}

// One-row task of a diagonal request with wide hub sums: the walks of start
// row k over edge records, <Q_k, C_h> for every requested active wide hub h
// next to k summed into hsumw (as k_diag_walk_wide does), then flushed.
template <class WT, bool DIGEST, bool CUTOFF>
__device__ void wide_row_task(const BReq &R, const WSeg &sg, int64_t rel, uint32_t k, uint2 rk, int32_t *vstate,
                              unsigned char *vxb, uint64_t &dig, unsigned long long &ns, double *hsumw,
                              uint32_t *hkw, double *red) {
    const int tid = threadIdx.x;
    const int64_t N = R.a.N;
    __syncthreads(); // the previous task is done with hkw and hsumw
    if (tid < kWideWords)
        hkw[tid] = 0u;
    __syncthreads();
    for (int hb = tid; hb < R.whub_act; hb += blockDim.x) {
        const bool adj = (R.wmask[int64_t(k) * kWideWords + hb / 32] >> (hb % 32)) & 1u;
        if (adj && (!R.a.in_set || R.a.in_set[R.whub_rows[hb]])) {
            atomicOr(&hkw[hb / 32], 1u << (hb % 32));
            hsumw[hb] = 0.0;
        }
    }
    __syncthreads();
    walk::WideRow hr;
    hr.chunks = 0u;
#pragma unroll
    for (int wd = 0; wd < kWideWords; ++wd) {
        hr.hk[wd] = static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(hkw[wd])));
        if (hr.hk[wd] != 0u)
            hr.chunks |= 1u << (wd >> 2);
    }
    hr.any = hr.chunks != 0u;
    const int64_t span = int64_t(R.a.K - 1) * N;
    WT *vx = reinterpret_cast<WT *>(vxb + sg.xoff) + rel * span;
    int32_t *vs = vstate + sg.slot_base + rel * span;
    double acc0 = 0.0;
    for (int64_t w = tid; w < N; w += blockDim.x) {
        uint64_t h = dev::kFnvBasis;
        walk::diag_walk_wide<WT, DIGEST, CUTOFF>(R.g.edge, reinterpret_cast<const uint4 *>(R.wmask), R.a, k, rk,
                                                 static_cast<uint32_t>(w), vs + w, vx + w, N, &h, &ns, hr, hsumw,
                                                 &acc0);
        dig += h;
    }
    if (hr.any) {
        const double x0 = dev::block_sum(acc0, red);
        for (int hb = tid; hb < R.whub_act; hb += blockDim.x) {
            if ((hkw[hb / 32] >> (hb % 32)) & 1u) {
                const double hs = hsumw[hb] + x0;
                if (hs != 0.0)
                    atomicAdd(&R.a.dacc[R.whub_rows[hb]], R.a.scale * (R.a.scale * hs) * (1.0 / static_cast<double>(N)));
            }
        }
    }
}

template <class WT, bool WEIGHTED, bool CUTOFF, bool DIGEST, bool VALUE, bool WIDE>
__global__ __launch_bounds__(kWalkThreads) void k_batch_walk(const BReq *__restrict__ reqs,
                                                             const WSeg *__restrict__ segs,
                                                             int n_segs, int64_t n_tasks,
                                                             int32_t *vstate, unsigned char *vxb,
                                                             unsigned long long *queue) {
    __shared__ double red[kWalkThreads / 64];
    __shared__ unsigned long long redu[kWalkThreads / 64];
    __shared__ double hsum[kHubRows * kMaxHubs]; // per row of the task, per hub
    __shared__ double hsumw[WIDE ? kMaxWideHubs : 1];
    __shared__ uint32_t hkw[WIDE ? kWideWords : 1];
    __shared__ int64_t task_slot;
    const int tid = threadIdx.x;
    // Tasks come from a queue counter in order, so the rows in flight stay a
    // narrow window of the task space (walks of neighbouring rows share cache
    // lines on graphs with locality).  The next task is claimed while the
    // current one runs.
    if (tid == 0)
        task_slot = static_cast<int64_t>(atomicAdd(queue, 1ull));
    __syncthreads();
    int64_t task = dev::uniform(task_slot);
    while (task < n_tasks) {
        unsigned long long next = 0;
        if (tid == 0)
            next = atomicAdd(queue, 1ull);
        int lo = 0, hi = n_segs;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segs[mid].task_base <= task)
                lo = mid;
            else
                hi = mid;
        }
        const WSeg &sg = segs[lo];
        const BReq &R = reqs[sg.req];
        const int64_t N = R.a.N;
        const int64_t local = task - sg.task_base;
        uint64_t h = dev::kFnvBasis;
        unsigned long long ns = 0;
        if (WIDE && sg.rows_per_task == 0) {
            // Wide hub sums (every task of a wide request is one row).
            const int64_t rel = local;
            const uint32_t k = static_cast<uint32_t>(dev::uniform(R.starts[sg.kk0 + rel]));
            const uint2 rk = R.g.node[k];
            uint64_t dig = 0;
            wide_row_task<WT, DIGEST, CUTOFF>(R, sg, rel, k, rk, vstate, vxb, dig, ns, hsumw, hkw, red);
            if (DIGEST) {
                const unsigned long long dg = dev::block_sum(static_cast<unsigned long long>(dig), redu);
                if (tid == 0)
                    atomicAdd(reinterpret_cast<unsigned long long *>(&R.digest[k]), dg);
            }
        } else if (sg.rows_per_task == 0) {
            // One row: every thread loops over its walks.
            const int64_t rel = local;
            const uint32_t k = static_cast<uint32_t>(dev::uniform(R.starts[sg.kk0 + rel]));
            const uint2 rk = R.g.node[k];
            // Diagonal requests: requested hubs adjacent to k are summed here.
            uint32_t hub_k = 0u;
            if constexpr (!WEIGHTED) {
                if (R.a.hub_act != 0u) {
                    hub_k = static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(R.g.hubmask[k]))) &
                            R.a.hub_act;
                    if (hub_k != 0u && R.a.in_set) {
                        const int lane = tid & 63;
                        const bool keep = lane < kMaxHubs && ((hub_k >> lane) & 1u) &&
                                          R.a.in_set[R.g.hub_row[lane]];
                        hub_k = static_cast<uint32_t>(__ballot(keep));
                    }
                    if (hub_k != 0u) {
                        if (tid < kMaxHubs)
                            hsum[tid] = 0.0;
                        __syncthreads();
                    }
                }
            }
            double acc = 0.0;
            uint64_t dig = 0;
            for (int64_t w = tid; w < N; w += blockDim.x) {
                h = dev::kFnvBasis;
                one_walk<WT, WEIGHTED, CUTOFF, DIGEST, VALUE>(R, sg, rel, k, rk, w, vstate, vxb, acc, h, ns,
                                                       hub_k, hsum);
                dig += h;
            }
            if (hub_k != 0u) {
                __syncthreads();
                if (tid < kMaxHubs && ((hub_k >> tid) & 1u) && hsum[tid] != 0.0)
                    atomicAdd(&R.a.dacc[R.g.hub_row[tid]],
                              R.a.scale * (R.a.scale * hsum[tid]) * (1.0 / static_cast<double>(N)));
                __syncthreads();
            }
            if (R.kind == MCMF_REQ_ACTION) {
                const double total = dev::block_sum(acc, red);
                if (tid == 0 && total != 0.0)
                    atomicAdd(&R.q[k], total / static_cast<double>(N));
            }
            if (DIGEST) {
                const unsigned long long dg = dev::block_sum(static_cast<unsigned long long>(dig), redu);
                if (tid == 0)
                    atomicAdd(reinterpret_cast<unsigned long long *>(&R.digest[k]), dg);
            }
        } else {
            // Several rows, one walk per thread.
            const int slot = tid / static_cast<int>(N);
            const int64_t rel = local * sg.rows_per_task + slot;
            const int64_t w = tid % N;
            const bool mine = tid < int64_t(sg.rows_per_task) * N && rel < sg.rows;
            // Diagonal requests with N >= kHubMinWalks: each row's requested
            // hubs are summed into its own slice of hsum.
            uint32_t hub_k = 0u;
            if constexpr (!WEIGHTED) {
                if (R.a.hub_act != 0u) {
                    if (mine) {
                        hub_k = R.g.hubmask[R.starts[sg.kk0 + rel]] & R.a.hub_act;
                        if (R.a.in_set) {
                            for (uint32_t m = hub_k; m != 0u; m &= m - 1u) {
                                const int b = __ffs(m) - 1;
                                if (!R.a.in_set[R.g.hub_row[b]])
                                    hub_k &= ~(1u << b);
                            }
                        }
                    }
                    for (int i = tid; i < kHubRows * kMaxHubs; i += blockDim.x)
                        hsum[i] = 0.0;
                    __syncthreads();
                }
            }
            if (mine) {
                const uint32_t k = static_cast<uint32_t>(R.starts[sg.kk0 + rel]);
                const uint2 rk = R.g.node[k];
                double acc = 0.0;
                one_walk<WT, WEIGHTED, CUTOFF, DIGEST, VALUE>(R, sg, rel, k, rk, w, vstate, vxb, acc, h, ns,
                                                       hub_k, hsum + slot * kMaxHubs);
                if (R.kind == MCMF_REQ_ACTION && acc != 0.0)
                    atomicAdd(&R.q[k], acc / static_cast<double>(N));
                if (DIGEST)
                    atomicAdd(reinterpret_cast<unsigned long long *>(&R.digest[k]),
                              static_cast<unsigned long long>(h));
            }
            if constexpr (!WEIGHTED) {
                if (R.a.hub_act != 0u) {
                    // Only bits of a row's hub_k were summed: a non-zero entry
                    // is a requested hub adjacent to that row.
                    __syncthreads();
                    for (int i = tid; i < kHubRows * kMaxHubs; i += blockDim.x)
                        if (hsum[i] != 0.0)
                            atomicAdd(&R.a.dacc[R.g.hub_row[i % kMaxHubs]],
                                      R.a.scale * (R.a.scale * hsum[i]) * (1.0 / static_cast<double>(N)));
                    __syncthreads();
                }
            }
        }
        const unsigned long long st = dev::block_sum(ns, redu);
        if (tid == 0) {
            atomicAdd(R.steps, st);
            task_slot = static_cast<int64_t>(next);
        }
        __syncthreads();
        task = dev::uniform(task_slot);
    }
}

using WalkKernel = void (*)(const BReq *, const WSeg *, int, int64_t, int32_t *, unsigned char *,
                            unsigned long long *);

template <int M>
WalkKernel walk_kernel_of() {
    using WT = typename std::conditional<(M & kModeFp32) != 0, float, double>::type;
    // The value mode exists only unweighted without a digest; the other
    // combinations never occur and share the plain kernel.
    constexpr bool kValue = (M & kModeValue) != 0 && (M & (kModeWeighted | kModeDigest)) == 0;
    constexpr bool kWide = (M & kModeWide) != 0 && (M & (kModeWeighted | kModeValue)) == 0;
    return &k_batch_walk<WT, (M & kModeWeighted) != 0, (M & kModeCutoff) != 0, (M & kModeDigest) != 0, kValue,
                         kWide>;
}

template <int... M>
WalkKernel walk_kernel_in(int m, std::integer_sequence<int, M...>) {
    WalkKernel table[] = {walk_kernel_of<M>()...};
    return table[m];
}

WalkKernel walk_kernel(int mode) {
    return walk_kernel_in(mode, std::make_integer_sequence<int, kWalkModes>{});
}

// Item bases of the runs of one gather launch (one thread; runs are few).
__global__ void k_seg_items(const BReq *__restrict__ reqs, GSeg *segs, int n_segs) {
    if (blockIdx.x != 0 || threadIdx.x != 0)
        return;
    int64_t base = 0;
    for (int i = 0; i < n_segs; ++i) {
        const int64_t *off = reqs[segs[i].req].item_off;
        segs[i].item_base = base;
        base += off[segs[i].kk0 + segs[i].rows] - off[segs[i].kk0];
    }
    segs[n_segs].item_base = base;
}

// The run and start row of every item of one gather launch, map[item] =
// {run, kk}, so that a workgroup finds them with one load instead of two
// binary searches.  One block row per run (blockIdx.y), one thread per start
// row; entries at or beyond cap are not written (the kernel searches).
__global__ void k_seg_item_rows(const BReq *__restrict__ reqs, const GSeg *__restrict__ segs, int2 *map,
                                int64_t cap) {
    const GSeg sg = segs[blockIdx.y];
    const int64_t rel = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (rel >= sg.rows)
        return;
    const int64_t *off = reqs[sg.req].item_off;
    const int64_t kk = sg.kk0 + rel;
    const int64_t first = sg.item_base - off[sg.kk0];
    for (int64_t it = off[kk]; it < off[kk + 1] && first + it < cap; ++it)
        map[first + it] = make_int2(static_cast<int>(blockIdx.y), static_cast<int>(kk));
}

template <bool WEIGHTED, class VT>
__global__ __launch_bounds__(gather::kGatherThreads) void k_batch_gather(
    const BReq *__restrict__ reqs, const GSeg *__restrict__ segs, int n_segs,
    const int32_t *vstate, const unsigned char *vxb, uint32_t nb, unsigned long long *probes_out,
    unsigned long long *queue, const int2 *__restrict__ map, int64_t map_cap) {
    using namespace gather;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Batch bt;
    __shared__ uint32_t scan_scratch[kWaves];
    __shared__ unsigned long long red[kWaves];
    __shared__ int64_t item_slot;
    const Shared sh = shared_views(smem, nb, &bt, scan_scratch, red);
    const int64_t n_items = segs[n_segs].item_base;
    unsigned long long probes = 0;
    for (;;) {
        const int64_t item = dev::uniform(next_item(queue, &item_slot));
        if (item >= n_items)
            break;
        int lo = 0;
        int64_t kk = -1;
        if (map && item < map_cap) {
            const int2 e = map[item];
            lo = dev::uniform(e.x);
            kk = dev::uniform(static_cast<int64_t>(e.y));
        } else {
            int hi = n_segs;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (segs[mid].item_base <= item)
                    lo = mid;
                else
                    hi = mid;
            }
        }
        const GSeg sg = segs[lo];
        const BReq &R = reqs[sg.req];
        const int64_t ri = dev::uniform(R.item_off[sg.kk0]) + (item - sg.item_base);
        if (kk < 0)
            kk = dev::uniform(row_of_item(R.item_off, sg.kk0, sg.kk0 + sg.rows, ri));
        const uint32_t part = static_cast<uint32_t>(ri - dev::uniform(R.item_off[kk]));
        const int64_t rel = kk - sg.kk0;
        const int64_t span = int64_t(R.a.K - 1) * R.a.N;
        RowJob job;
        job.k = dev::uniform(R.starts[kk]);
        const uint2 rk = R.g.node[job.k];
        job.rk = make_uint2(static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(rk.x))),
                            static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(rk.y))));
        job.p_begin = part * R.item;
        job.p_end = job.rk.y - job.p_begin < R.item ? job.rk.y : job.p_begin + R.item;
        job.st = vstate + sg.slot_base + rel * span;
        job.N = R.a.N;
        job.K = R.a.K;
        job.walks_per_pass = R.wpp;
        job.node = R.g.node;
        job.col = R.g.col;
        job.val = R.g.val;
        job.in_set = R.in_set;
        job.scale = R.a.scale;
        job.dacc = R.dacc;
        job.overflow = probes_out + 1;
        job.hub_of = R.hub_of;
        job.hub_act = R.hub_act;
        job.whub_of = R.whub_of;
        job.whub_act = R.whub_act;
        gather_row<WEIGHTED, VT>(sh, job, reinterpret_cast<const VT *>(vxb + sg.xoff) + rel * span,
                                 probes);
    }
    const unsigned long long total = dev::block_sum(probes, red);
    if (threadIdx.x == 0)
        atomicAdd(probes_out, total);
}

// Gather kernel for variant v = (FP32 weights ? 1 : 0) | (weighted ? 2 : 0).
using GatherKernel = void (*)(const BReq *, const GSeg *, int, const int32_t *,
                              const unsigned char *, uint32_t, unsigned long long *,
                              unsigned long long *, const int2 *, int64_t);
constexpr int kGatherVariants = 4;
GatherKernel gather_kernel(int v) {
    switch (v) {
    case 0: return &k_batch_gather<false, double>;
    case 1: return &k_batch_gather<false, float>;
    case 2: return &k_batch_gather<true, double>;
    default: return &k_batch_gather<true, float>;
    }
}

// Host-side state of one request.
struct Prep {
    mcmf_request *req = nullptr;
    std::vector<double> c;
    DevBuf<double> coef, r, q, dacc;
    DevBuf<uint4> rec; // action value records (when used)
    DevBuf<uint8_t> in_set, start_flags;
    DevBuf<int32_t> start_list;
    DevBuf<int64_t> items;
    const int64_t *item_off = nullptr;
    View<double> vin, out;
    View<int32_t> rows;
    View<uint64_t> dig;
    const int32_t *starts = nullptr;
    int64_t n_start = 0;
    int64_t count = 0; // outputs
    bool all = false;
};

} // namespace

Status check_request(mcmf_request &q) {
    mcmf_opts o = {};
    o.precision = q.precision;
    o.weight_cutoff = q.weight_cutoff;
    MCMF_TRY(check_common(q.graph, &q.fn, q.n_walks, q.K, &o));
    if (!q.out)
        return fail(MCMF_E_ARG, "request output is NULL");
    if (q.kind == MCMF_REQ_ACTION) {
        if (!q.v)
            return fail(MCMF_E_ARG, "action request without v");
        if (q.v == q.out)
            return fail(MCMF_E_ARG, "out may not alias v");
    } else if (q.kind == MCMF_REQ_DIAG) {
        if (!q.graph->symmetric)
            return fail(MCMF_E_NOT_SYMMETRIC, "diag request on a graph not created with MCMF_SYMMETRIC");
        if (q.rows && q.n_rows < 0)
            return fail(MCMF_E_ARG, "n_rows is negative");
    } else {
        return fail(MCMF_E_ARG, "unknown request kind %d", q.kind);
    }
    return {};
}

namespace {

// value_budget: bytes of action value records the batch may still hold.
Status prepare(Prep &P, hipStream_t s, uint64_t *value_budget) {
    mcmf_request &q = *P.req;
    const mcmf_graph *g = q.graph;
    const int64_t n = g->n;
    P.c.resize(q.K + 1);
    MCMF_TRY(make_coeffs(&q.fn, q.K, P.c.data()));
    if (q.K >= 2) {
        MCMF_TRY(P.coef.alloc(q.K - 1, s));
        MCMF_HIP(hipMemcpyAsync(P.coef.ptr, P.c.data() + 2, sizeof(double) * (q.K - 1),
                                hipMemcpyHostToDevice, s));
    }
    if (q.path_digest) {
        MCMF_TRY(P.dig.out(q.path_digest, n, s));
    }
    if (q.kind == MCMF_REQ_ACTION) {
        P.count = n;
        MCMF_TRY(P.vin.in(q.v, n, s));
        MCMF_TRY(P.out.out(q.out, n, s));
        MCMF_TRY(P.r.alloc(n > 0 ? n : 1, s));
        MCMF_TRY(spmv_r(g, P.vin.ptr, q.fn.scale, P.r.ptr, s));
        if (q.K >= 2) {
            MCMF_TRY(P.q.alloc(n > 0 ? n : 1, s));
            P.starts = g->active;
            P.n_start = g->n_active;
            // Value records when the graph's tuning asks for them (as a single
            // call would) and the batch's share of memory allows.
            const uint64_t bytes = static_cast<uint64_t>(g->nnz) * sizeof(uint4);
            if (g->tuning.action_sampler == MCMF_SAMPLER_VALUE && !g->weighted && !q.path_digest &&
                g->nnz > 0 && bytes <= *value_budget) {
                MCMF_TRY(P.rec.alloc(g->nnz, s));
                MCMF_TRY(build_value_records(g, P.r.ptr, P.rec.ptr, s));
                *value_budget -= bytes;
            }
        }
        return {};
    }
    P.all = q.rows == nullptr;
    P.count = P.all ? n : q.n_rows;
    MCMF_TRY(P.out.out(q.out, P.count, s));
    if (!P.all) {
        MCMF_TRY(P.rows.in(q.rows, P.count, s));
        MCMF_TRY(P.in_set.alloc(n > 0 ? n : 1, s));
        MCMF_TRY(fill_u8(P.in_set.ptr, 0, n, s));
        DevBuf<int> bad;
        MCMF_TRY(bad.alloc(1, s));
        MCMF_TRY(fill_i32(bad.ptr, 0, 1, s));
        MCMF_TRY(mark_rows(P.rows.ptr, P.count, n, P.in_set.ptr, bad.ptr, s));
        int hbad = 0;
        MCMF_HIP(hipMemcpyAsync(&hbad, bad.ptr, sizeof hbad, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipStreamSynchronize(s));
        if (hbad)
            return fail(MCMF_E_ARG, "a requested row lies outside [0, %lld)", static_cast<long long>(n));
    }
    if (q.K >= 2) {
        MCMF_TRY(P.dacc.alloc(n > 0 ? n : 1, s));
        if (P.all) {
            P.starts = g->active;
            P.n_start = g->n_active;
            P.item_off = g->active_items;
        } else if (P.count > 0) {
            MCMF_TRY(P.start_flags.alloc(n > 0 ? n : 1, s));
            MCMF_TRY(P.start_list.alloc(n > 0 ? n : 1, s));
            MCMF_TRY(fill_u8(P.start_flags.ptr, 0, n, s));
            MCMF_TRY(mark_starts(g, P.rows.ptr, P.count, P.start_flags.ptr, s));
            MCMF_TRY(compact(P.start_flags.ptr, n, 1, P.start_list.ptr, &P.n_start, s));
            P.starts = P.start_list.ptr;
            MCMF_TRY(P.items.alloc(P.n_start + 1, s));
            MCMF_TRY(gather_items(g, P.starts, P.n_start, P.items.ptr, s));
            P.item_off = P.items.ptr;
        }
    }
    return {};
}

} // namespace

Status run_batch(mcmf_request *reqs, int64_t n_reqs, const mcmf_batch_opts *o, mcmf_stats *stats) {
    if (n_reqs < 0 || (n_reqs > 0 && !reqs))
        return fail(MCMF_E_ARG, "bad request array");
    if (o) {
        if (o->reserved0)
            return fail(MCMF_E_ARG, "reserved option words must be zero");
        for (uint32_t r : o->reserved)
            if (r)
                return fail(MCMF_E_ARG, "reserved option words must be zero");
    }
    for (int64_t i = 0; i < n_reqs; ++i)
        reqs[i].status = MCMF_OK;
    for (int64_t i = 0; i < n_reqs; ++i) {
        Status st = check_request(reqs[i]);
        if (st) {
            reqs[i].status = st.code;
            return st;
        }
    }
    if (n_reqs == 0)
        return {};
    const int device = reqs[0].graph->device;
    for (int64_t i = 0; i < n_reqs; ++i)
        if (reqs[i].graph->device != device)
            return fail(MCMF_E_ARG, "all requests of a batch must use graphs on one device");
    MCMF_HIP(hipSetDevice(device));
    hipStream_t s = (o && o->stream) ? static_cast<hipStream_t>(o->stream) : reqs[0].graph->stream;
    const bool use_graph = o && o->use_graph;

    std::vector<std::unique_ptr<Prep>> preps(n_reqs);
    uint64_t value_budget = device_memory_bytes() / 16; // action value records of the whole batch
    for (int64_t i = 0; i < n_reqs; ++i) {
        preps[i].reset(new Prep());
        preps[i]->req = &reqs[i];
        Status st = prepare(*preps[i], s, &value_budget);
        if (st) {
            reqs[i].status = st.code;
            return st;
        }
    }

    // Descriptors.
    std::vector<BReq> hreq(n_reqs);
    for (int64_t i = 0; i < n_reqs; ++i) {
        const mcmf_request &q = reqs[i];
        Prep &P = *preps[i];
        BReq &B = hreq[i];
        memset(&B, 0, sizeof B);
        B.g = walk::view(q.graph, (q.kind == MCMF_REQ_DIAG ? q.graph->tuning.diag_sampler
                                                            : q.graph->tuning.action_sampler) == MCMF_SAMPLER_ALIAS);
        mcmf_opts oo = {};
        oo.seed = q.seed;
        oo.request_id = q.request_id;
        oo.precision = q.precision;
        oo.weight_cutoff = q.weight_cutoff;
        B.a = walk::to_args(walk_params(&oo, P.coef.ptr, q.K, q.fn.scale, q.n_walks));
        B.kind = q.kind;
        B.mode = (q.precision == MCMF_PRECISION_FP32_WEIGHTS ? kModeFp32 : 0) |
                 (q.graph->weighted ? kModeWeighted : 0) | (q.weight_cutoff > 0.0 ? kModeCutoff : 0) |
                 (P.dig.ptr ? kModeDigest : 0) | (P.rec.ptr ? kModeValue : 0);
        B.rec = P.rec.ptr;
        B.starts = P.starts;
        B.r = P.r.ptr;
        B.q = P.q.ptr;
        B.digest = P.dig.ptr;
        B.in_set = P.all ? nullptr : P.in_set.ptr;
        B.dacc = P.dacc.ptr;
        B.item_off = P.item_off;
        B.item = gather_item(q.graph);
        if (q.kind == MCMF_REQ_DIAG && !q.graph->weighted && q.n_walks >= kRowTaskWalks &&
            q.graph->n_whubs > 0 &&
            (q.graph->tuning.diag_sampler == MCMF_SAMPLER_WIDE ||
             (q.graph->tuning.diag_sampler == MCMF_SAMPLER_AUTO && auto_wide(q.graph, q.n_walks, q.K)))) {
            // Wide hub rows (one start row per task): the walks sum them, the
            // gather leaves them out.
            B.mode |= kModeWide;
            B.wmask = q.graph->wmask;
            B.whub_rows = q.graph->whub_rows;
            B.whub_of = q.graph->whub_of;
            B.whub_act = active_wide_hubs(q.graph, q.n_walks, q.K);
            B.a.in_set = B.in_set;
            B.a.dacc = B.dacc;
        } else if (q.kind == MCMF_REQ_DIAG && !q.graph->weighted && q.n_walks >= kHubMinWalks) {
            // Hub rows: the walks sum them, the gather leaves them out.
            B.hub_of = q.graph->hub_of;
            B.hub_act = active_hubs(q.graph, q.n_walks, q.K);
            B.a.hub_act = B.hub_act;
            B.a.in_set = B.in_set;
            B.a.dacc = B.dacc;
        }
    }
    DevBuf<unsigned long long> counters; // per request steps, then probes, overflow
    MCMF_TRY(counters.alloc(n_reqs + 2, s));
    for (int64_t i = 0; i < n_reqs; ++i)
        hreq[i].steps = counters.ptr + i;

    // Gather plan of each diagonal request: its own table size (so a request
    // with few walks keeps a small table and many workgroups per CU) and
    // walks per pass.
    const size_t table_lds = gather::kMaxTableLds;
    std::vector<uint32_t> req_nb(n_reqs, 0);
    std::vector<size_t> req_lds(n_reqs, 0);
    for (int64_t i = 0; i < n_reqs; ++i) {
        const mcmf_request &q = reqs[i];
        if (q.kind != MCMF_REQ_DIAG || q.K < 2 || preps[i]->n_start == 0)
            continue;
        GatherPlan plan = plan_gather(q.graph->n, q.n_walks, q.K, table_lds,
                                      sizeof(uint32_t) * gather::kFilterWords, gather::kSlots);
        if (!plan.ok)
            return fail(MCMF_E_UNSUPPORTED, "no Q_k table layout fits LDS for N=%lld, K=%d",
                        static_cast<long long>(q.n_walks), q.K);
        hreq[i].wpp = plan.walks_per_pass;
        req_nb[i] = static_cast<uint32_t>(plan.cap / gather::kSlots);
        req_lds[i] = plan.lds_bytes;
    }
    DevBuf<BReq> dreq;
    MCMF_TRY(dreq.alloc(n_reqs, s));
    MCMF_HIP(hipMemcpyAsync(dreq.ptr, hreq.data(), sizeof(BReq) * n_reqs, hipMemcpyHostToDevice, s));

    // Launch plan: chunk 0 = every action task + the first diag rows; later
    // chunks = diag rows only.  Each chunk holds at most `budget` bytes of
    // visit records.  Walk runs are kept per walk-kernel variant, gather runs
    // per (gather variant, table size): one launch each.
    int64_t budget = default_visit_chunk_bytes();
    if (o && o->visit_chunk_bytes)
        budget = static_cast<int64_t>(std::min<uint64_t>(o->visit_chunk_bytes, uint64_t(1) << 62));
    struct GatherGroup {
        int variant;
        uint32_t nb;
        size_t lds;
        std::vector<GSeg> segs;
    };
    struct Chunk {
        std::vector<WSeg> w[kWalkModes];
        int64_t tasks[kWalkModes] = {};
        std::vector<GatherGroup> g;
        int64_t rows = 0, slots = 0, xbytes = 0;
    };
    auto add_walks = [&](Chunk &c, int64_t i, int64_t kk0, int64_t rows, int64_t slot_base, int64_t xoff) {
        const int m = hreq[i].mode;
        const int64_t N = reqs[i].n_walks;
        WSeg w = {};
        w.req = static_cast<int32_t>(i);
        w.kk0 = kk0;
        w.rows = rows;
        w.task_base = c.tasks[m];
        w.slot_base = slot_base;
        w.xoff = xoff;
        int64_t tasks;
        if (N >= kRowTaskWalks) {
            w.rows_per_task = 0;
            tasks = rows;
        } else {
            w.rows_per_task = static_cast<uint32_t>(kWalkThreads / N);
            tasks = (rows + w.rows_per_task - 1) / w.rows_per_task;
        }
        c.w[m].push_back(w);
        c.tasks[m] += tasks;
    };
    std::vector<Chunk> chunks(1);
    for (int64_t i = 0; i < n_reqs; ++i) {
        const mcmf_request &q = reqs[i];
        if (q.kind != MCMF_REQ_ACTION || q.K < 2 || preps[i]->n_start == 0)
            continue;
        add_walks(chunks[0], i, 0, preps[i]->n_start, 0, 0);
    }
    for (int64_t i = 0; i < n_reqs; ++i) {
        const mcmf_request &q = reqs[i];
        if (q.kind != MCMF_REQ_DIAG || q.K < 2 || preps[i]->n_start == 0)
            continue;
        const int64_t span = q.n_walks * (q.K - 1);
        const int64_t xb = q.precision == MCMF_PRECISION_FP32_WEIGHTS ? 4 : 8;
        const int64_t row_bytes = span * (4 + xb);
        const int var = (q.precision == MCMF_PRECISION_FP32_WEIGHTS ? 1 : 0) | (q.graph->weighted ? 2 : 0);
        int64_t kk = 0;
        while (kk < preps[i]->n_start) {
            Chunk &c = chunks.back();
            const int64_t used = c.slots * 4 + c.xbytes + 8;
            int64_t fit = (budget - used) / row_bytes;
            if (fit < 1 && c.rows > 0) {
                chunks.emplace_back();
                continue;
            }
            fit = std::max<int64_t>(fit, 1);
            const int64_t take = std::min(fit, preps[i]->n_start - kk);
            // Value arrays are 8-byte aligned per run.
            c.xbytes = (c.xbytes + 7) & ~int64_t(7);
            add_walks(c, i, kk, take, c.slots, c.xbytes);
            GatherGroup *grp = nullptr;
            for (auto &gg : c.g)
                if (gg.variant == var && gg.nb == req_nb[i])
                    grp = &gg;
            if (!grp) {
                c.g.push_back(GatherGroup{var, req_nb[i], req_lds[i], {}});
                grp = &c.g.back();
            }
            grp->segs.push_back(GSeg{static_cast<int32_t>(i), kk, take, 0, c.slots, c.xbytes});
            c.rows += take;
            c.slots += take * span;
            c.xbytes += take * span * xb;
            kk += take;
        }
    }
    int64_t max_slots = 0, max_xbytes = 0;
    for (const Chunk &c : chunks) {
        max_slots = std::max(max_slots, c.slots);
        max_xbytes = std::max(max_xbytes, c.xbytes);
    }
    DevBuf<int32_t> vstate;
    DevBuf<unsigned char> vxb;
    MCMF_TRY(vstate.alloc(max_slots > 0 ? max_slots : 1, s));
    MCMF_TRY(vxb.alloc(max_xbytes > 0 ? max_xbytes : 8, s));
    // Device copies of the run tables; the gather table of a group carries a
    // spare entry for its item count.
    std::vector<std::unique_ptr<DevBuf<WSeg>>> dws;
    std::vector<std::unique_ptr<DevBuf<GSeg>>> dgs;
    // Item maps of the gather launches (k_seg_item_rows), sized from the
    // runs (item_map_entries per run, at most kMaxItemMap in all).  Launches
    // with more runs than a grid's second dimension holds search instead.
    std::vector<std::unique_ptr<DevBuf<int2>>> dmaps;
    std::vector<int64_t> map_caps, map_rows;
    size_t lds_max[kGatherVariants] = {0, 0, 0, 0};
    int64_t n_groups = 0;
    for (const Chunk &c : chunks) {
        for (int m = 0; m < kWalkModes; ++m) {
            dws.emplace_back(new DevBuf<WSeg>());
            if (c.w[m].empty())
                continue;
            MCMF_TRY(dws.back()->alloc(c.w[m].size(), s));
            MCMF_HIP(hipMemcpyAsync(dws.back()->ptr, c.w[m].data(), sizeof(WSeg) * c.w[m].size(),
                                    hipMemcpyHostToDevice, s));
        }
        for (const GatherGroup &gg : c.g) {
            dgs.emplace_back(new DevBuf<GSeg>());
            MCMF_TRY(dgs.back()->alloc(gg.segs.size() + 1, s));
            MCMF_HIP(hipMemcpyAsync(dgs.back()->ptr, gg.segs.data(), sizeof(GSeg) * gg.segs.size(),
                                    hipMemcpyHostToDevice, s));
            lds_max[gg.variant] = std::max(lds_max[gg.variant], gg.lds);
            int64_t cap = 0, most_rows = 0;
            for (const GSeg &sg : gg.segs) {
                const mcmf_graph *sgg = reqs[sg.req].graph;
                cap = std::min(kMaxItemMap,
                               cap + item_map_entries(sg.rows, sgg->nnz, sgg->d_max, hreq[sg.req].item));
                most_rows = std::max(most_rows, sg.rows);
            }
            dmaps.emplace_back(new DevBuf<int2>());
            cap = item_map_cap(cap);
            if (gg.segs.size() > 65535u || most_rows == 0)
                cap = 0;
            if (cap > 0)
                MCMF_TRY(dmaps.back()->alloc(cap, s));
            map_caps.push_back(cap);
            map_rows.push_back(most_rows);
            ++n_groups;
        }
    }
    for (int v = 0; v < kGatherVariants; ++v)
        if (lds_max[v] > 0)
            MCMF_TRY(gather::allow_table_lds(reinterpret_cast<const void *>(gather_kernel(v))));
    // Persistent gather workgroups per group: as many as fit at once.
    std::vector<int64_t> group_blocks;
    for (const Chunk &c : chunks)
        for (const GatherGroup &gg : c.g) {
            int per_cu = 0;
            MCMF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &per_cu, reinterpret_cast<const void *>(gather_kernel(gg.variant)), gather::kGatherThreads,
                gg.lds));
            group_blocks.push_back(int64_t(per_cu > 0 ? per_cu : 1) * num_cus());
        }
    // One work counter per gather launch, then one per (chunk, walk mode).
    const int64_t walk_queue0 = n_groups;
    const int64_t n_queues = n_groups + static_cast<int64_t>(chunks.size()) * kWalkModes;
    DevBuf<unsigned long long> queues;
    MCMF_TRY(queues.alloc(n_queues, s));

    // Walk workgroups: exactly as many as are resident at once.  The tasks
    // are dealt out in order, so the device works through a narrow window of
    // the task space (one or two requests, one graph's data in the caches);
    // workgroups waiting for a slot would start at the front of the task
    // space and spread the window over every request.
    int64_t walk_blocks[kWalkModes] = {};
    for (const Chunk &c : chunks)
        for (int m = 0; m < kWalkModes; ++m)
            if (c.tasks[m] > 0 && walk_blocks[m] == 0) {
                int per_cu = 0;
                MCMF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(
                    &per_cu, reinterpret_cast<const void *>(walk_kernel(m)), kWalkThreads, 0));
                walk_blocks[m] = int64_t(per_cu > 0 ? per_cu : 1) * num_cus();
            }

    // The device work of the batch: fills, walks, gathers, assembly.
    auto enqueue = [&](hipStream_t es) -> Status {
        MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(counters.ptr), 0, n_reqs + 2, es));
        MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(queues.ptr), 0, n_queues, es));
        for (int64_t i = 0; i < n_reqs; ++i) {
            Prep &P = *preps[i];
            const int64_t n = reqs[i].graph->n;
            if (P.q.ptr)
                MCMF_TRY(fill_f64(P.q.ptr, 0.0, n, es));
            if (P.dacc.ptr)
                MCMF_TRY(fill_f64(P.dacc.ptr, 0.0, n, es));
            if (P.dig.ptr)
                MCMF_TRY(fill_u64(P.dig.ptr, 0, n, es));
        }
        int64_t gi = 0;
        for (size_t ci = 0; ci < chunks.size(); ++ci) {
            const Chunk &c = chunks[ci];
            for (int m = 0; m < kWalkModes; ++m) {
                if (c.tasks[m] == 0)
                    continue;
                const int64_t blocks = std::min<int64_t>(walk_blocks[m], c.tasks[m]);
                hipLaunchKernelGGL(walk_kernel(m), dim3(static_cast<uint32_t>(blocks)), dim3(kWalkThreads), 0,
                                   es, dreq.ptr, dws[ci * kWalkModes + m]->ptr, static_cast<int>(c.w[m].size()),
                                   c.tasks[m], vstate.ptr, vxb.ptr,
                                   queues.ptr + walk_queue0 + static_cast<int64_t>(ci) * kWalkModes + m);
                MCMF_HIP(hipGetLastError());
            }
            for (const GatherGroup &gg : c.g) {
                GSeg *segs = dgs[gi]->ptr;
                const int n_segs = static_cast<int>(gg.segs.size());
                hipLaunchKernelGGL(k_seg_items, dim3(1), dim3(64), 0, es, dreq.ptr, segs, n_segs);
                MCMF_HIP(hipGetLastError());
                if (map_caps[gi] > 0) {
                    hipLaunchKernelGGL(k_seg_item_rows,
                                       dim3(static_cast<uint32_t>((map_rows[gi] + 255) / 256),
                                            static_cast<uint32_t>(n_segs)),
                                       dim3(256), 0, es, dreq.ptr, segs, dmaps[gi]->ptr, map_caps[gi]);
                    MCMF_HIP(hipGetLastError());
                }
                hipLaunchKernelGGL(gather_kernel(gg.variant), dim3(static_cast<uint32_t>(group_blocks[gi])),
                                   dim3(gather::kGatherThreads), gg.lds, es, dreq.ptr, segs, n_segs,
                                   vstate.ptr, vxb.ptr, gg.nb, counters.ptr + n_reqs, queues.ptr + gi,
                                   map_caps[gi] > 0 ? dmaps[gi]->ptr : nullptr, map_caps[gi]);
                MCMF_HIP(hipGetLastError());
                ++gi;
            }
        }
        for (int64_t i = 0; i < n_reqs; ++i) {
            const mcmf_request &q = reqs[i];
            Prep &P = *preps[i];
            const double c1 = q.K >= 1 ? P.c[1] : 0.0;
            if (q.kind == MCMF_REQ_ACTION)
                MCMF_TRY(spmv_assemble(q.graph, P.vin.ptr, P.r.ptr, q.K >= 2 ? P.q.ptr : nullptr,
                                       P.c[0], c1, q.fn.scale, P.out.ptr, es));
            else
                MCMF_TRY(diag_finish(q.graph, P.all ? nullptr : P.rows.ptr, P.count, q.K, P.c[0], c1,
                                     q.fn.scale, P.dacc.ptr, P.out.ptr, es));
        }
        return {};
    };

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
        MCMF_HIP(hipEventCreate(&e0));
        MCMF_HIP(hipEventCreate(&e1));
        MCMF_HIP(hipEventRecord(e0, s));
    }
    if (use_graph) {
        // Record on a stream of the batch's own: a capture that fails leaves
        // its stream unusable on this runtime (still marked as an invalidated
        // capture after hipStreamEndCapture), so the caller's stream never
        // enters capture mode; the graph is launched on it.
        hipStream_t cs = nullptr;
        MCMF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        const hipError_t be = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        // Test hook: the capture "fails" before its first launch (MCMF_TEST_FAIL_CAPTURE=1).
        const char *refuse = getenv("MCMF_TEST_FAIL_CAPTURE");
        const Status st = be != hipSuccess ? hip_fail(be, "hipStreamBeginCapture", __FILE__, __LINE__)
                          : refuse && refuse[0] == '1'
                              ? fail(MCMF_E_DEVICE, "capture refused (MCMF_TEST_FAIL_CAPTURE)")
                              : enqueue(cs);
        const hipError_t ce = be == hipSuccess ? hipStreamEndCapture(cs, &graph) : hipSuccess;
        if (st || ce != hipSuccess) {
            // The capture failed.  Another host thread can make a call that
            // invalidates captures in progress; the runtime reports it at the
            // next launch being recorded or at the end of the capture.
            // Nothing captured has run: run the batch's launches directly on
            // the caller's stream instead (a genuine error then shows again,
            // and is returned).
            (void)hipGetLastError();
            if (graph)
                (void)hipGraphDestroy(graph);
            (void)hipStreamDestroy(cs);
            (void)hipGetLastError();
            clear_error();
            MCMF_TRY(enqueue(s));
        } else {
            (void)hipStreamDestroy(cs);
            hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                (void)hipGraphDestroy(graph);
                MCMF_HIP(ie);
            }
            hipError_t le = hipGraphLaunch(exec, s);
            hipError_t se = hipStreamSynchronize(s);
            (void)hipGraphExecDestroy(exec);
            (void)hipGraphDestroy(graph);
            MCMF_HIP(le);
            MCMF_HIP(se);
        }
    } else {
        MCMF_TRY(enqueue(s));
    }
    if (stats)
        MCMF_HIP(hipEventRecord(e1, s));

    // Results back to host buffers; counters.
    for (int64_t i = 0; i < n_reqs; ++i) {
        Prep &P = *preps[i];
        MCMF_TRY(P.out.copy_back(reqs[i].out, P.count, s));
        if (reqs[i].path_digest)
            MCMF_TRY(P.dig.copy_back(reqs[i].path_digest, reqs[i].graph->n, s));
    }
    std::vector<unsigned long long> hc(n_reqs + 2, 0);
    MCMF_HIP(hipMemcpyAsync(hc.data(), counters.ptr, sizeof(unsigned long long) * (n_reqs + 2),
                            hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    if (hc[n_reqs + 1] != 0)
        return fail(MCMF_E_DEVICE, "internal error: a Q_k table overflowed (%llu inserts lost)",
                    hc[n_reqs + 1]);
    uint64_t steps = 0, walks = 0, starts = 0;
    for (int64_t i = 0; i < n_reqs; ++i) {
        reqs[i].walk_steps = hc[i];
        steps += hc[i];
        if (reqs[i].K >= 2) {
            starts += preps[i]->n_start;
            walks += preps[i]->n_start * reqs[i].n_walks;
        }
    }
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->start_rows = starts;
        stats->walks = walks;
        stats->walk_steps = steps;
        stats->gather_probes = hc[n_reqs];
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            (void)hipGetLastError();
        stats->ms_total = ms;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
    }
    return {};
}

} // namespace mcmf

extern "C" mcmf_status mcmf_batch(mcmf_request *reqs, int64_t n_reqs, const mcmf_batch_opts *opts,
                                  mcmf_stats *stats) {
    mcmf::clear_error();
    return mcmf::run_batch(reqs, n_reqs, opts, stats).code;
}
