// RandFunmAction (Section 3.4, Algorithm 3):
//   r = s A v                         (one sparse product)
//   q_k from the walks                (walk.hip)
//   y = c0 v + c1 r + s A q            (one sparse product, Eq. rand_funm_action_formula)
//
// The sparse products group rows by length: rows of at most 64 entries use
// 8 lanes per row, rows of at most 4096 entries a wavefront, longer rows a
// 1024-thread workgroup.  Every row's sum is reduced in a fixed order.
#include <vector>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

constexpr int kShortLanes = 8;

enum class Out { Records, Assemble };

// Row sum s * sum_j a_ij x_j by a group of G lanes; every lane of the group
// gets the total.
template <int G, bool WEIGHTED>
__device__ __forceinline__ double row_dot(const int32_t *__restrict__ col,
                                          const double *__restrict__ val,
                                          const double *__restrict__ x, uint32_t start,
                                          uint32_t deg, int lane_in_group) {
    double sum = 0.0;
    for (uint32_t e = lane_in_group; e < deg; e += G) {
        const int64_t idx = int64_t(start) + e;
        const double xv = x[col[idx]];
        sum += WEIGHTED ? val[idx] * xv : xv;
    }
    return dev::group_sum<G>(sum);
}

struct SpmvArgs {
    const uint2 *node;
    const int32_t *col;
    const double *val;
    const int32_t *rows; // this bin's rows
    int64_t count;
    const double *x;     // v (records) or q (assemble)
    double scale;
    // Records: r out
    double *rout;
    // Assemble
    const double *v;
    const double *rin;
    double c0, c1;
    double *y;
};

template <Out OUT>
__device__ __forceinline__ void emit(const SpmvArgs &a, int32_t i, uint2 nd, double dot) {
    if (OUT == Out::Records) {
        a.rout[i] = a.scale * dot;
    } else {
        double yi = a.c0 * a.v[i] + a.c1 * a.rin[i];
        if (a.x)
            yi += a.scale * dot;
        a.y[i] = yi;
    }
}

// Groups of G lanes, one row per group (G = 8 or 64).
template <int G, bool WEIGHTED, Out OUT>
__global__ __launch_bounds__(256) void k_spmv_groups(SpmvArgs a) {
    const int lane_in_group = threadIdx.x & (G - 1);
    const int64_t groups = int64_t(gridDim.x) * (blockDim.x / G);
    for (int64_t r = blockIdx.x * int64_t(blockDim.x / G) + threadIdx.x / G; r < a.count;
         r += groups) {
        const int32_t i = a.rows[r];
        const uint2 nd = a.node[i];
        double dot = 0.0;
        if (a.x)
            dot = row_dot<G, WEIGHTED>(a.col, a.val, a.x, nd.x, nd.y, lane_in_group);
        if (lane_in_group == 0)
            emit<OUT>(a, i, nd, dot);
    }
}

// One 1024-thread workgroup per long row.
template <bool WEIGHTED, Out OUT>
__global__ __launch_bounds__(1024) void k_spmv_long(SpmvArgs a) {
    __shared__ double red[16];
    for (int64_t r = blockIdx.x; r < a.count; r += gridDim.x) {
        const int32_t i = a.rows[r];
        const uint2 nd = a.node[i];
        double sum = 0.0;
        if (a.x) {
            for (uint32_t e = threadIdx.x; e < nd.y; e += blockDim.x) {
                const int64_t idx = int64_t(nd.x) + e;
                const double xv = a.x[a.col[idx]];
                sum += WEIGHTED ? a.val[idx] * xv : xv;
            }
        }
        const double dot = dev::block_sum(sum, red);
        if (threadIdx.x == 0)
            emit<OUT>(a, i, nd, dot);
        __syncthreads();
    }
}

int64_t cap_grid(int64_t blocks) {
    const int64_t cap = int64_t(1) << 20;
    return blocks < 1 ? 1 : (blocks < cap ? blocks : cap);
}

template <Out OUT>
Status launch_spmv(const mcmf_graph *g, SpmvArgs a, hipStream_t s) {
    a.node = g->node;
    a.col = g->col;
    a.val = g->val;
    const bool w = g->weighted;
    for (int b = 0; b < 3; ++b) {
        a.rows = g->bin_rows + g->bin_offset[b];
        a.count = g->bin_count[b];
        if (a.count == 0)
            continue;
        if (b == 0) {
            const dim3 grid(cap_grid((a.count + 256 / kShortLanes - 1) / (256 / kShortLanes)));
            if (w)
                hipLaunchKernelGGL((k_spmv_groups<kShortLanes, true, OUT>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_spmv_groups<kShortLanes, false, OUT>), grid, dim3(256), 0, s, a);
        } else if (b == 1) {
            const dim3 grid(cap_grid((a.count + 3) / 4));
            if (w)
                hipLaunchKernelGGL((k_spmv_groups<64, true, OUT>), grid, dim3(256), 0, s, a);
            else
                hipLaunchKernelGGL((k_spmv_groups<64, false, OUT>), grid, dim3(256), 0, s, a);
        } else {
            const dim3 grid(cap_grid(a.count));
            if (w)
                hipLaunchKernelGGL((k_spmv_long<true, OUT>), grid, dim3(1024), 0, s, a);
            else
                hipLaunchKernelGGL((k_spmv_long<false, OUT>), grid, dim3(1024), 0, s, a);
        }
        MCMF_HIP(hipGetLastError());
    }
    return {};
}

} // namespace

Status spmv_r(const mcmf_graph *g, const double *v, double scale, double *r, hipStream_t s) {
    SpmvArgs a = {};
    a.x = v;
    a.scale = scale;
    a.rout = r;
    return launch_spmv<Out::Records>(g, a, s);
}

Status spmv_assemble(const mcmf_graph *g, const double *v, const double *rec, const double *q,
                     double c0, double c1, double scale, double *y, hipStream_t s) {
    SpmvArgs a = {};
    a.x = q;
    a.scale = scale;
    a.v = v;
    a.rin = rec;
    a.c0 = c0;
    a.c1 = c1;
    a.y = y;
    return launch_spmv<Out::Assemble>(g, a, s);
}

} // namespace mcmf
