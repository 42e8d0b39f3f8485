// Diagonal gather kernel of the single-request path.  Work items are
// neighbour ranges of start rows (at most 256 neighbours each, so a hub row
// is spread over many workgroups); persistent workgroups take items from a
// queue counter and run gather::gather_row (gather_core.hpp) on each.
#include <hip/hip_runtime.h>

#include "gather_core.hpp"

namespace mcmf {

namespace {

using namespace gather;

__global__ void k_item_counts(const int32_t *__restrict__ starts, int64_t n,
                              const uint2 *__restrict__ node, uint32_t item, uint32_t *__restrict__ cnt) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n)
        cnt[i] = items_of(node[starts[i]].y, item);
}

// Exclusive prefix sums of cnt[0..n) into off[0..n], one workgroup of 1024
// threads, 8 counts per thread per tile.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;
__global__ __launch_bounds__(kScanThreads) void k_item_scan(const uint32_t *__restrict__ cnt,
                                                            int64_t n, int64_t *__restrict__ off) {
    __shared__ uint32_t scratch[kScanThreads / 64];
    int64_t carry = 0;
    const int64_t tile = int64_t(kScanThreads) * kScanPer;
    for (int64_t t0 = 0; t0 < n; t0 += tile) {
        const int64_t base = t0 + int64_t(threadIdx.x) * kScanPer;
        uint32_t v[kScanPer];
        uint32_t local = 0;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            v[u] = base + u < n ? cnt[base + u] : 0u;
            local += v[u];
        }
        uint32_t total = 0;
        const uint32_t before = dev::block_exclusive_scan(local, scratch, &total);
        int64_t run = carry + before;
#pragma unroll
        for (int u = 0; u < kScanPer; ++u) {
            if (base + u < n)
                off[base + u] = run;
            run += v[u];
        }
        carry += total;
        __syncthreads(); // scratch is reused by the next tile
    }
    if (threadIdx.x == 0)
        off[n] = carry;
}

// Start row of each work item of one gather launch: item_row[it - off[lo]]
// = kk for every item it of start row kk in [lo, hi), so that a workgroup
// finds its row with one load instead of a binary search over off (one
// dependent global load per level, paid by every item).  Entries beyond cap
// are not written; the kernel searches for those.
__global__ void k_item_rows(const int64_t *__restrict__ off, int64_t lo, int64_t hi,
                            int32_t *__restrict__ item_row, int64_t cap) {
    const int64_t kk = lo + int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (kk >= hi)
        return;
    const int64_t base = off[lo];
    const int64_t e = off[kk + 1];
    for (int64_t it = off[kk]; it < e && it - base < cap; ++it)
        item_row[it - base] = static_cast<int32_t>(kk);
}

struct GatherArgs {
    const int32_t *item_row; // k_item_rows of this launch
    int64_t item_cap;        // entries of item_row
    const uint2 *node;
    const int32_t *col;
    const double *val;
    const int32_t *starts;
    const int64_t *item_off;
    int64_t row_begin, row_end;
    int64_t N;
    int K;
    int64_t walks_per_pass;
    const int32_t *vstate; // records of start row row_begin onwards
    const void *vx;        // double[] or float[] (FP32 walk weights)
    const uint8_t *in_set; // null: every row requested
    const int32_t *row_walks; // per start row (whole start list); null: N each
    const int64_t *row_rec;   // first visit record per start row (with row_walks)
    double scale;
    uint32_t nb; // buckets
    double *dacc;
    unsigned long long *probes;
    unsigned long long *overflow; // set if a table ever fills (a planning error)
    unsigned long long *queue;
    const uint8_t *hub_of;
    uint32_t hub_act; // hubs the walks summed: left out of the probes
    uint32_t item;    // neighbours per work item
    const uint16_t *whub_of;
    int32_t whub_act; // wide hubs the walks summed (prefix): left out too
};

template <bool WEIGHTED, class VT>
__global__ __launch_bounds__(kGatherThreads) void k_diag_gather(GatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Batch bt;
    __shared__ uint32_t scan_scratch[kWaves];
    __shared__ unsigned long long red[kWaves];
    __shared__ int64_t item_slot[2];
    const Shared sh = shared_views(smem, a.nb, &bt, scan_scratch, red);
    const int64_t span = int64_t(a.K - 1) * a.N;
    const int64_t first = a.item_off[a.row_begin];
    const int64_t last = a.item_off[a.row_end];
    unsigned long long probes = 0;
    RowJob job;
    job.N = a.N;
    job.K = a.K;
    job.walks_per_pass = a.walks_per_pass;
    job.node = a.node;
    job.col = a.col;
    job.val = a.val;
    job.in_set = a.in_set;
    job.scale = a.scale;
    job.dacc = a.dacc;
    job.overflow = a.overflow;
    job.hub_of = a.hub_of;
    job.hub_act = a.hub_act;
    job.whub_of = a.whub_of;
    job.whub_act = a.whub_act;
    // The queue counter of the next item is fetched while the current one
    // runs.
    // Two slots: thread 0 writes the next item's at the end of an item, while
    // the other threads may still be reading the current one's.
    unsigned long long next = 0;
    if (threadIdx.x == 0)
        item_slot[0] = static_cast<int64_t>(atomicAdd(a.queue, 1ull));
    for (int64_t it = 0;; ++it) {
        __syncthreads(); // the slot is written; every thread is done with the previous item
        const int64_t item = dev::uniform(first + item_slot[it & 1]);
        if (item >= last)
            break;
        if (threadIdx.x == 0)
            next = atomicAdd(a.queue, 1ull);
        const int64_t kk = item - first < a.item_cap
                               ? dev::uniform(static_cast<int64_t>(a.item_row[item - first]))
                               : dev::uniform(row_of_item(a.item_off, a.row_begin, a.row_end, item));
        const uint32_t part = static_cast<uint32_t>(item - dev::uniform(a.item_off[kk]));
        job.k = dev::uniform(a.starts[kk]);
        const uint2 rk = a.node[job.k];
        job.rk = make_uint2(static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(rk.x))),
                            static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(rk.y))));
        job.p_begin = part * a.item;
        job.p_end = job.rk.y - job.p_begin < a.item ? job.rk.y : job.p_begin + a.item;
        int64_t rec = (kk - a.row_begin) * span;
        if (a.row_walks) {
            job.N = dev::uniform(static_cast<int64_t>(a.row_walks[kk]));
            rec = dev::uniform(a.row_rec[kk] - a.row_rec[a.row_begin]);
        }
        job.st = a.vstate + rec;
        gather_row<WEIGHTED, VT>(sh, job, static_cast<const VT *>(a.vx) + rec, probes);
        if (threadIdx.x == 0)
            item_slot[(it + 1) & 1] = static_cast<int64_t>(next);
    }
    if (a.probes) {
        const unsigned long long total = dev::block_sum(probes, red);
        if (threadIdx.x == 0)
            atomicAdd(a.probes, total);
    }
}

} // namespace

uint32_t gather_item(const mcmf_graph *g) {
    return static_cast<uint32_t>(g->tuning.gather_item > 0 ? g->tuning.gather_item : kDefaultGatherItem);
}

Status refresh_active_items(mcmf_graph *g) {
    MCMF_HIP(hipSetDevice(g->device));
    MCMF_TRY(gather_items(g, g->active, g->n_active, g->active_items, g->stream));
    MCMF_HIP(hipStreamSynchronize(g->stream));
    return {};
}

Status gather_items(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t *off,
                    hipStream_t s, uint32_t item) {
    if (n_start < 0)
        return fail(MCMF_E_ARG, "negative start-row count");
    DevBuf<uint32_t> cnt;
    MCMF_TRY(cnt.alloc(n_start > 0 ? n_start : 1, s));
    if (n_start > 0) {
        const int64_t blocks = (n_start + 255) / 256;
        hipLaunchKernelGGL(k_item_counts, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, starts,
                           n_start, g->node, item ? item : gather_item(g), cnt.ptr);
        MCMF_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_item_scan, dim3(1), dim3(kScanThreads), 0, s, cnt.ptr, n_start, off);
    MCMF_HIP(hipGetLastError());
    return {};
}

Status diag_gather(const mcmf_graph *g, const int32_t *starts, const int64_t *item_off,
                   int64_t row_begin, int64_t row_end, const WalkParams &p, const int32_t *state,
                   const void *x, const uint8_t *in_set, double *dacc, unsigned long long *probes,
                   unsigned long long *overflow, unsigned long long *queue, hipStream_t s) {
    if (row_end <= row_begin || p.K < 2)
        return {};
    GatherArgs a = {};
    a.node = g->node;
    a.col = g->col;
    a.val = g->val;
    a.starts = starts;
    a.item_off = item_off;
    a.row_begin = row_begin;
    a.row_end = row_end;
    a.N = p.n_walks;
    a.K = p.K;
    a.vstate = state;
    a.vx = x;
    a.in_set = in_set;
    a.row_walks = p.row_walks;
    a.row_rec = p.row_rec;
    a.scale = p.scale;
    a.dacc = dacc;
    a.probes = probes;
    a.queue = queue;
    a.hub_of = g->hub_of;
    a.hub_act = p.hub_act;
    a.whub_of = g->whub_of;
    a.whub_act = wide_diag(g, p) ? p.whub_act : 0;
    a.item = p.gather_item ? p.gather_item : gather_item(g);
    DevBuf<int32_t> item_rows;
    a.item_cap = item_map_cap(item_map_entries(row_end - row_begin, g->nnz, g->d_max, a.item));
    MCMF_TRY(item_rows.alloc(a.item_cap > 0 ? a.item_cap : 1, s));
    hipLaunchKernelGGL(k_item_rows, dim3(static_cast<uint32_t>((row_end - row_begin + 255) / 256)), dim3(256), 0, s,
                       item_off, row_begin, row_end, item_rows.ptr, a.item_cap);
    MCMF_HIP(hipGetLastError());
    a.item_row = item_rows.ptr;
    const GatherPlan plan = plan_gather(g->n, p.n_walks, p.K, kMaxTableLds,
                                        sizeof(uint32_t) * kFilterWords, kSlots);
    if (!plan.ok)
        return fail(MCMF_E_UNSUPPORTED, "no Q_k table layout fits LDS for N=%lld, K=%d",
                    static_cast<long long>(p.n_walks), p.K);
    a.nb = static_cast<uint32_t>(plan.cap / kSlots);
    a.walks_per_pass = plan.walks_per_pass;
    a.overflow = overflow;
    const size_t lds = plan.lds_bytes;
    const bool fp32 = p.precision == MCMF_PRECISION_FP32_WEIGHTS;
    auto launch = [&](auto kernel) -> Status {
        const void *fn = reinterpret_cast<const void *>(kernel);
        MCMF_TRY(allow_table_lds(fn));
        // Persistent workgroups: as many as fit on the device at once.
        int per_cu = 0;
        MCMF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kGatherThreads, lds));
        const int64_t blocks = int64_t(per_cu > 0 ? per_cu : 1) * num_cus();
        hipLaunchKernelGGL(kernel, dim3(static_cast<uint32_t>(blocks)), dim3(kGatherThreads), lds, s, a);
        return {};
    };
    if (g->weighted)
        MCMF_TRY(fp32 ? launch(&k_diag_gather<true, float>) : launch(&k_diag_gather<true, double>));
    else
        MCMF_TRY(fp32 ? launch(&k_diag_gather<false, float>) : launch(&k_diag_gather<false, double>));
    MCMF_HIP(hipGetLastError());
    return {};
}

} // namespace mcmf
