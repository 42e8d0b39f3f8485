// Diagonal gather kernel of the single-request path: one 1024-thread
// workgroup per start row; the per-row work is gather::gather_row
// (gather_core.hpp).
#include "gather_core.hpp"

namespace mcmf {

namespace {

using namespace gather;

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
    const void *vx; // double[] or float[] (FP32 walk weights)
    const uint8_t *in_set; // null: every row requested
    double scale;
    uint32_t nb; // buckets
    double *dacc;
    unsigned long long *probes;
    unsigned long long *overflow; // set if a table ever fills (a planning error)
};

template <bool WEIGHTED, class VT>
__global__ __launch_bounds__(kGatherThreads) void k_diag_gather(GatherArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ Batch bt;
    __shared__ uint32_t scan_scratch[kWaves];
    __shared__ unsigned long long red[kWaves];
    const Shared sh = shared_views(smem, a.nb, &bt, scan_scratch, red);
    const int64_t span = int64_t(a.K - 1) * a.N;
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
    for (int64_t kk = blockIdx.x; kk < a.n_start; kk += gridDim.x) {
        job.k = a.starts[kk];
        job.rk = a.node[job.k];
        job.st = a.vstate + kk * span;
        gather_row<WEIGHTED, VT>(sh, job, static_cast<const VT *>(a.vx) + kk * span, probes);
    }
    if (a.probes) {
        const unsigned long long total = dev::block_sum(probes, red);
        if (threadIdx.x == 0)
            atomicAdd(a.probes, total);
    }
}

} // namespace

Status diag_gather(const mcmf_graph *g, const int32_t *starts, int64_t n_start, const WalkParams &p,
                   const int32_t *state, const void *x, const uint8_t *in_set, double *dacc,
                   unsigned long long *probes, unsigned long long *overflow, hipStream_t s) {
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
    const GatherPlan plan = plan_gather(g->n, p.n_walks, p.K, 160 * 1024 - kStaticLds,
                                        sizeof(uint32_t) * kFilterWords, kSlots);
    if (!plan.ok)
        return fail(MCMF_E_UNSUPPORTED, "no Q_k table layout fits LDS for N=%lld, K=%d",
                    static_cast<long long>(p.n_walks), p.K);
    a.nb = static_cast<uint32_t>(plan.cap / kSlots);
    a.walks_per_pass = plan.walks_per_pass;
    a.overflow = overflow;
    const size_t lds = plan.lds_bytes;
    const int64_t cap_blocks = int64_t(1) << 20;
    const dim3 grid(static_cast<uint32_t>(n_start < cap_blocks ? n_start : cap_blocks));
    const bool fp32 = p.precision == MCMF_PRECISION_FP32_WEIGHTS;
    auto launch = [&](auto kernel) -> Status {
        MCMF_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds)));
        hipLaunchKernelGGL(kernel, grid, dim3(kGatherThreads), lds, s, a);
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
