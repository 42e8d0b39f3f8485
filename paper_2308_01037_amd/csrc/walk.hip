// Walk kernels of the single-request path (Lemma 2; Algorithm 3 for the
// action, Eq. rand_funm_Q for the diagonal).  One workgroup per start row k
// runs that row's walks; lane w runs walk w (and w + blockDim, ...).  The walk
// itself is in walk_core.hpp.
#include <algorithm>

#include "walk_core.hpp"

namespace mcmf {

namespace {

using walk::GraphView;
using walk::WalkArgs;

// Action: q[k] = (1/N) sum_w sum_t c_{t+2} W_t r_{l_t}.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF, bool EDGE, bool STREAM>
__global__ __launch_bounds__(256) void k_action_walk(GraphView g, const double *__restrict__ r,
                                                     const int32_t *__restrict__ starts,
                                                     int64_t n_start, WalkArgs a,
                                                     double *__restrict__ q,
                                                     uint64_t *__restrict__ digest,
                                                     unsigned long long *steps) {
    __shared__ double red[4];
    __shared__ unsigned long long redu[4];
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = g.node[k];
        const double r_k = r[k];
        const int64_t N = a.row_walks ? a.row_walks[kk] : a.N;
        double acc = 0.0;
        uint64_t dig = 0;
        unsigned long long nsteps = 0;
        for (int64_t w64 = threadIdx.x; w64 < N; w64 += blockDim.x) {
            uint64_t h = dev::kFnvBasis;
            acc += walk::action_walk<WT, WEIGHTED, DIGEST, CUTOFF, EDGE, STREAM>(
                g, r, a, k, rk, r_k, static_cast<uint32_t>(w64), &h, &nsteps);
            if (DIGEST)
                dig += h;
        }
        const double total = dev::block_sum(acc, red);
        const unsigned long long st = dev::block_sum(nsteps, redu);
        if (DIGEST) {
            const unsigned long long dg = dev::block_sum(static_cast<unsigned long long>(dig), redu);
            if (threadIdx.x == 0)
                digest[k] = dg;
        }
        if (threadIdx.x == 0) {
            q[k] = total / static_cast<double>(N);
            if (steps)
                atomicAdd(steps, st);
        }
    }
}

// Diagonal: visit records of start row kk, t-major: slot (kk*(K-1) + t)*N + w
// holds (l_t, c_{t+2} W_t); after a walk ends early its slots hold state -1.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF, bool EDGE, bool STREAM>
__global__ __launch_bounds__(256) void k_diag_walk(GraphView g, const int32_t *__restrict__ starts,
                                                   int64_t n_start, WalkArgs a,
                                                   int32_t *__restrict__ vstate,
                                                   WT *__restrict__ vx,
                                                   uint64_t *__restrict__ digest,
                                                   unsigned long long *steps) {
    __shared__ unsigned long long redu[4];
    __shared__ double hsum[kMaxHubs];
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = g.node[k];
        const int64_t N = a.row_walks ? a.row_walks[kk] : a.N;
        const int64_t row_base = a.row_rec ? a.row_rec[kk] - a.row_rec[0] : kk * (a.K - 1) * a.N;
        // Requested hubs adjacent to k: their <Q_k, C_h> are summed here.
        uint32_t hub_k = 0u;
        if constexpr (!WEIGHTED) {
            if (a.hub_act != 0u) {
                hub_k = static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(g.hubmask[k]))) & a.hub_act;
                if (hub_k != 0u && a.in_set) {
                    const int lane = threadIdx.x & 63;
                    const bool keep = lane < kMaxHubs && ((hub_k >> lane) & 1u) && a.in_set[g.hub_row[lane]];
                    hub_k = static_cast<uint32_t>(__ballot(keep));
                }
                if (hub_k != 0u) {
                    if (threadIdx.x < kMaxHubs)
                        hsum[threadIdx.x] = 0.0;
                    __syncthreads();
                }
            }
        }
        uint64_t dig = 0;
        unsigned long long nsteps = 0;
        for (int64_t w64 = threadIdx.x; w64 < N; w64 += blockDim.x) {
            uint64_t h = dev::kFnvBasis;
            walk::diag_walk<WT, WEIGHTED, DIGEST, CUTOFF, EDGE, STREAM>(g, a, k, rk, static_cast<uint32_t>(w64),
                                                           vstate + row_base + w64,
                                                           vx + row_base + w64, N, &h, &nsteps,
                                                           hub_k, hsum);
            if (DIGEST)
                dig += h;
        }
        if (hub_k != 0u) {
            // dacc[h] += s a_kh * s <Q_k, C_h> / N, as the gather adds it.
            __syncthreads();
            const int t = threadIdx.x;
            if (t < kMaxHubs && ((hub_k >> t) & 1u) && hsum[t] != 0.0)
                atomicAdd(&a.dacc[g.hub_row[t]], a.scale * (a.scale * hsum[t]) * (1.0 / static_cast<double>(N)));
            __syncthreads();
        }
        const unsigned long long st = dev::block_sum(nsteps, redu);
        if (DIGEST) {
            const unsigned long long dg = dev::block_sum(static_cast<unsigned long long>(dig), redu);
            if (threadIdx.x == 0)
                digest[k] = dg;
        }
        if (threadIdx.x == 0 && steps)
            atomicAdd(steps, st);
    }
}

// Diagonal with wide hub sums (unweighted graphs): the visit records as
// k_diag_walk writes them, and <Q_k, C_h> for every requested wide hub h of
// the active prefix [0, n_act) adjacent to k summed here (the gather leaves
// those neighbours out): dacc[h] += s a_kh * s <Q_k, C_h> / N.
template <class WT, bool DIGEST, bool CUTOFF>
__global__ __launch_bounds__(256) void k_diag_walk_wide(const uint2 *__restrict__ node,
                                                        const uint4 *__restrict__ edge,
                                                        const uint32_t *__restrict__ wmask,
                                                        const int32_t *__restrict__ whub_rows, int32_t n_act,
                                                        const int32_t *__restrict__ starts, int64_t n_start,
                                                        WalkArgs a, int32_t *__restrict__ vstate,
                                                        WT *__restrict__ vx, uint64_t *__restrict__ digest,
                                                        unsigned long long *steps) {
    __shared__ unsigned long long redu[4];
    __shared__ double redd[4];
    __shared__ double hsum[kMaxWideHubs];
    __shared__ uint32_t hk[kWideWords];
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = node[k];
        const int64_t N = a.row_walks ? a.row_walks[kk] : a.N;
        const int64_t row_base = a.row_rec ? a.row_rec[kk] - a.row_rec[0] : kk * (a.K - 1) * a.N;
        // The requested active hubs adjacent to k.
        __syncthreads();
        if (threadIdx.x < kWideWords)
            hk[threadIdx.x] = 0u;
        __syncthreads();
        for (int hb = threadIdx.x; hb < n_act; hb += blockDim.x) {
            const bool adj = (wmask[int64_t(k) * kWideWords + hb / 32] >> (hb % 32)) & 1u;
            if (adj && (!a.in_set || a.in_set[whub_rows[hb]])) {
                atomicOr(&hk[hb / 32], 1u << (hb % 32));
                hsum[hb] = 0.0;
            }
        }
        __syncthreads();
        walk::WideRow hr;
        hr.chunks = 0u;
#pragma unroll
        for (int wd = 0; wd < kWideWords; ++wd) {
            hr.hk[wd] = static_cast<uint32_t>(dev::uniform(static_cast<int32_t>(hk[wd])));
            if (hr.hk[wd] != 0u)
                hr.chunks |= 1u << (wd >> 2);
        }
        hr.any = hr.chunks != 0u;
        uint64_t dig = 0;
        unsigned long long nsteps = 0;
        double acc0 = 0.0;
        for (int64_t w64 = threadIdx.x; w64 < N; w64 += blockDim.x) {
            uint64_t h = dev::kFnvBasis;
            walk::diag_walk_wide<WT, DIGEST, CUTOFF>(edge, reinterpret_cast<const uint4 *>(wmask), a, k, rk,
                                                     static_cast<uint32_t>(w64),
                                                     vstate + row_base + w64, vx + row_base + w64, N, &h,
                                                     &nsteps, hr, hsum, &acc0);
            if (DIGEST)
                dig += h;
        }
        if (hr.any) {
            const double x0 = dev::block_sum(acc0, redd);
            for (int hb = threadIdx.x; hb < n_act; hb += blockDim.x) {
                if ((hk[hb / 32] >> (hb % 32)) & 1u) {
                    const double hs = hsum[hb] + x0;
                    if (hs != 0.0)
                        atomicAdd(&a.dacc[whub_rows[hb]], a.scale * (a.scale * hs) * (1.0 / static_cast<double>(N)));
                }
            }
        }
        const unsigned long long st = dev::block_sum(nsteps, redu);
        if (DIGEST) {
            const unsigned long long dg = dev::block_sum(static_cast<unsigned long long>(dig), redu);
            if (threadIdx.x == 0)
                digest[k] = dg;
        }
        if (threadIdx.x == 0 && steps)
            atomicAdd(steps, st);
    }
}

// Action over value records (unweighted graphs, no path digest).
template <class WT, bool CUTOFF, bool STREAM>
__global__ __launch_bounds__(256) void k_action_walk_value(const uint2 *__restrict__ node,
                                                           const uint4 *__restrict__ rec,
                                                           const double *__restrict__ r,
                                                           const int32_t *__restrict__ starts,
                                                           int64_t n_start, WalkArgs a,
                                                           double *__restrict__ q,
                                                           unsigned long long *steps) {
    __shared__ double red[4];
    __shared__ unsigned long long redu[4];
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = node[k];
        const double r_k = r[k];
        const int64_t N = a.row_walks ? a.row_walks[kk] : a.N;
        double acc = 0.0;
        unsigned long long nsteps = 0;
        for (int64_t w64 = threadIdx.x; w64 < N; w64 += blockDim.x)
            acc += walk::action_walk_value<WT, CUTOFF, STREAM>(rec, a, k, rk, r_k,
                                                               static_cast<uint32_t>(w64), &nsteps);
        const double total = dev::block_sum(acc, red);
        const unsigned long long st = dev::block_sum(nsteps, redu);
        if (threadIdx.x == 0) {
            q[k] = total / static_cast<double>(N);
            if (steps)
                atomicAdd(steps, st);
        }
    }
}

// rec[e] = {first entry of row col[e], its length, r[col[e]]} from the edge
// records.
__global__ void k_value_records(const uint4 *__restrict__ edge, int64_t nnz, const double *__restrict__ r,
                                uint4 *__restrict__ rec) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nnz;
         e += int64_t(gridDim.x) * blockDim.x) {
        const uint4 x = edge[e];
        const double v = r[x.x];
        rec[e] = make_uint4(x.y, x.z, static_cast<uint32_t>(__double2loint(v)),
                            static_cast<uint32_t>(__double2hiint(v)));
    }
}

// Lanes per start row: the walk count rounded up to whole wavefronts, at most
// 256, or fewer when the tuning (or the call) asks for fewer.
int walk_block(int64_t N, int threads) {
    int b = N >= 256 ? 256 : static_cast<int>(((N + 63) / 64) * 64);
    if (threads > 0 && threads < b)
        b = threads;
    return b;
}

// Workgroups loop over start rows, so the grid stays within the 32-bit
// work-item count of a dispatch whatever the number of start rows.
dim3 walk_grid(int64_t n_start) {
    const int64_t cap = int64_t(1) << 22;
    return dim3(static_cast<uint32_t>(n_start < cap ? n_start : cap));
}

} // namespace

bool value_records_fit(const mcmf_graph *g) {
    return static_cast<uint64_t>(g->nnz) * sizeof(uint4) <= device_memory_bytes() / 16;
}

Status build_value_records(const mcmf_graph *g, const double *r, uint4 *rec, hipStream_t s) {
    if (g->nnz <= 0)
        return {};
    const int64_t blocks = std::min<int64_t>((g->nnz + 255) / 256, int64_t(1) << 20);
    hipLaunchKernelGGL(k_value_records, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, g->edge, g->nnz,
                       r, rec);
    MCMF_HIP(hipGetLastError());
    return {};
}

Status action_walks(const mcmf_graph *g, const double *r, const int32_t *starts, int64_t n_start,
                    const WalkParams &p, double *q, uint64_t *digest, unsigned long long *steps,
                    hipStream_t s) {
    if (n_start <= 0 || p.K < 2)
        return {};
    const WalkArgs a = walk::to_args(p);
    const int sampler = p.sampler >= 0 ? p.sampler : g->tuning.action_sampler;
    const GraphView gv = walk::view(g, sampler == MCMF_SAMPLER_ALIAS);
    const int threads = p.threads >= 0 ? p.threads : g->tuning.walk_threads;
    const dim3 grid = walk_grid(n_start), block(p.row_walks ? 256 : walk_block(p.n_walks, threads));
    const bool stream = (p.stream >= 0 ? p.stream : g->tuning.action_stream) != 0;
    if (sampler == MCMF_SAMPLER_VALUE && !g->weighted && !digest && value_records_fit(g)) {
        DevBuf<uint4> rec;
        MCMF_TRY(rec.alloc(g->nnz, s));
        MCMF_TRY(build_value_records(g, r, rec.ptr, s));
        const bool fp32 = p.precision == MCMF_PRECISION_FP32_WEIGHTS;
        const bool cut = p.cutoff > 0.0;
        auto launch = [&](auto kernel) {
            hipLaunchKernelGGL(kernel, grid, block, 0, s, g->node, rec.ptr, r, starts, n_start, a, q, steps);
        };
        if (fp32)
            cut ? (stream ? launch(k_action_walk_value<float, true, true>) : launch(k_action_walk_value<float, true, false>))
                : (stream ? launch(k_action_walk_value<float, false, true>) : launch(k_action_walk_value<float, false, false>));
        else
            cut ? (stream ? launch(k_action_walk_value<double, true, true>) : launch(k_action_walk_value<double, true, false>))
                : (stream ? launch(k_action_walk_value<double, false, true>) : launch(k_action_walk_value<double, false, false>));
        MCMF_HIP(hipGetLastError());
        return {};
    }
    const bool edge = sampler != MCMF_SAMPLER_ROW;
    walk::dispatch6(p.precision == MCMF_PRECISION_FP32_WEIGHTS, g->weighted, digest != nullptr,
                    p.cutoff > 0.0, edge, stream, [&](auto wt, auto w, auto d, auto c, auto e, auto st) {
                        using WT = decltype(wt);
                        hipLaunchKernelGGL((k_action_walk<WT, decltype(w)::value, decltype(d)::value,
                                                          decltype(c)::value, decltype(e)::value,
                                                          decltype(st)::value>),
                                           grid, block, 0, s, gv, r, starts, n_start, a, q, digest,
                                           steps);
                    });
    MCMF_HIP(hipGetLastError());
    return {};
}

bool wide_diag(const mcmf_graph *g, const WalkParams &p) {
    if (g->n_whubs == 0 || g->weighted)
        return false;
    const int s = p.sampler >= 0 ? p.sampler : g->tuning.diag_sampler;
    return s == MCMF_SAMPLER_WIDE || (s == MCMF_SAMPLER_AUTO && auto_wide(g, p.n_walks, p.K));
}

Status diag_walks(const mcmf_graph *g, const int32_t *starts, int64_t n_start, const WalkParams &p,
                  int32_t *state, void *x, uint64_t *digest, unsigned long long *steps,
                  hipStream_t s) {
    if (n_start <= 0 || p.K < 2)
        return {};
    const WalkArgs a = walk::to_args(p);
    const GraphView gv =
        walk::view(g, (p.sampler >= 0 ? p.sampler : g->tuning.diag_sampler) == MCMF_SAMPLER_ALIAS);
    const int threads = p.threads >= 0 ? p.threads : g->tuning.walk_threads;
    const dim3 grid = walk_grid(n_start), block(p.row_walks ? 256 : walk_block(p.n_walks, threads));
    if (wide_diag(g, p)) {
        const bool fp32 = p.precision == MCMF_PRECISION_FP32_WEIGHTS;
        walk::dispatch4(fp32, false, digest != nullptr, p.cutoff > 0.0, [&](auto wt, auto, auto d, auto c) {
            using WT = decltype(wt);
            hipLaunchKernelGGL((k_diag_walk_wide<WT, decltype(d)::value, decltype(c)::value>), grid, block, 0, s,
                               g->node, g->edge, g->wmask, g->whub_rows, p.whub_act, starts, n_start, a, state,
                               static_cast<WT *>(x), digest, steps);
        });
        MCMF_HIP(hipGetLastError());
        return {};
    }
    const bool edge = (p.sampler >= 0 ? p.sampler : g->tuning.diag_sampler) != MCMF_SAMPLER_ROW;
    const bool stream = (p.stream >= 0 ? p.stream : g->tuning.diag_stream) != 0;
    walk::dispatch6(p.precision == MCMF_PRECISION_FP32_WEIGHTS, g->weighted, digest != nullptr,
                    p.cutoff > 0.0, edge, stream, [&](auto wt, auto w, auto d, auto c, auto e, auto st) {
                        using WT = decltype(wt);
                        hipLaunchKernelGGL((k_diag_walk<WT, decltype(w)::value, decltype(d)::value,
                                                        decltype(c)::value, decltype(e)::value,
                                                        decltype(st)::value>),
                                           grid, block, 0, s, gv, starts, n_start, a, state,
                                           static_cast<WT *>(x), digest, steps);
                    });
    MCMF_HIP(hipGetLastError());
    return {};
}

} // namespace mcmf
