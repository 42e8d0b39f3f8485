// Random-walk kernels of the estimator (Lemma 2; Algorithm 3 for the action,
// Eq. rand_funm_Q for the diagonal).  One workgroup per start row k runs
// that row's walks; lane w runs walk w (and w + blockDim, ...).
//
// A walk keeps its state in registers: the current row l with its record
// (first entry, length) and the weight W.  Per recorded step t it either adds
// c_{t+2} W r_l to a register sum (action) or writes the visit
// (l, c_{t+2} W) to the visit buffer (diagonal).  A transition draws
// Philox4x32-10 at counter (k, w, t, request), picks entry j of row l and
// moves to its column, multiplying W by s * sum_j |a_lj| (negated for a
// negative entry).
//
// Unweighted rows pick j = floor(u deg / 2^64) and read one 16-byte edge
// record {next row, its first entry, its length}: one dependent load per
// step.  The transition of step t is issued before step t is recorded, so
// the record's load overlaps the bookkeeping; the action's r_l load sits off
// that dependency chain.  Weighted rows search the running sums of |a|.
//
// Weight type WT: double (FP64 path) or float (FP32 walk weights).  With
// float, W, the per-step factor s * sum|a| and each row contribution
// c_{t+2} W r_l (action) or visit value c_{t+2} W (diagonal) are FP32; the
// sums over steps, walks and the gather stay FP64.  Paths are identical in
// both modes (sampling is integer), so the difference is rounding only.
#include <type_traits>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

// First index j < deg with target < cum[j] (cum non-decreasing); deg-1 if none.
__device__ __forceinline__ uint32_t cdf_search(const double *__restrict__ cum, uint32_t deg,
                                               double target) {
    uint32_t lo = 0, hi = deg;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (target < cum[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo < deg ? lo : deg - 1;
}

struct WalkArgs {
    const double *coef; // c_{t+2} at index t
    int K;
    double scale;
    int64_t N;
    uint32_t key0, key1, request;
    double cutoff;
};

WalkArgs to_args(const WalkParams &p) {
    WalkArgs a;
    a.coef = p.coef;
    a.K = p.K;
    a.scale = p.scale;
    a.N = p.n_walks;
    a.key0 = p.key0;
    a.key1 = p.key1;
    a.request = p.request;
    a.cutoff = p.cutoff;
    return a;
}

struct GraphView {
    const uint2 *node;
    const uint4 *edge;
    const int32_t *col;
    const double *val;
    const double *rowabs;
    const double *cum;
};

GraphView view(const mcmf_graph *g) {
    GraphView v;
    v.node = g->node;
    v.edge = g->edge;
    v.col = g->col;
    v.val = g->val;
    v.rowabs = g->rowabs;
    v.cum = g->cum;
    return v;
}

// Walk state of one walk: row, its record, weight.
struct Pos {
    uint32_t l, start, deg;
};

// One transition out of row p (deg > 0) with the block of random words x.
// Updates W (times s * sum |a|, sign of the entry) and returns the new row.
template <bool WEIGHTED, class WT>
__device__ __forceinline__ Pos step(const GraphView &g, const Pos &p, uint4 x, double scale,
                                    WT &W) {
    Pos n;
    if constexpr (!WEIGHTED) {
        const uint32_t j = dev::uniform_index(x.x, x.y, p.deg);
        W = W * static_cast<WT>(scale * static_cast<double>(p.deg));
        const uint4 e = g.edge[int64_t(p.start) + j];
        n.l = e.x;
        n.start = e.y;
        n.deg = e.z;
    } else {
        const double ra = g.rowabs[p.l];
        const uint32_t j = cdf_search(g.cum + p.start, p.deg, dev::unit53(x.x, x.y) * ra);
        W = W * static_cast<WT>(scale * ra);
        if (g.val[int64_t(p.start) + j] < 0.0)
            W = -W;
        n.l = static_cast<uint32_t>(g.col[int64_t(p.start) + j]);
        const uint2 r = g.node[n.l];
        n.start = r.x;
        n.deg = r.y;
    }
    return n;
}

// Action: q[k] = (1/N) sum_w sum_t c_{t+2} W_t r_{l_t}.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF>
__global__ __launch_bounds__(256) void k_action_walk(GraphView g, const double *__restrict__ r,
                                                     const int32_t *__restrict__ starts,
                                                     int64_t n_start, WalkArgs a,
                                                     double *__restrict__ q,
                                                     uint64_t *__restrict__ digest,
                                                     unsigned long long *steps) {
    __shared__ double red[4];
    __shared__ unsigned long long redu[4];
    const int last = a.K - 2;
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = g.node[k];
        const double r_k = r[k];
        double acc = 0.0;
        uint64_t dig = 0;
        unsigned long long nsteps = 0;
        for (int64_t w64 = threadIdx.x; w64 < a.N; w64 += blockDim.x) {
            const uint32_t w = static_cast<uint32_t>(w64);
            Pos p{k, rk.x, rk.y};
            double rl = r_k;
            WT W = WT(1);
            double wacc = 0.0;
            uint64_t h = dev::kFnvBasis;
            for (int t = 0; t <= last; ++t) {
                if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
                    break;
                const bool more = t < last && p.deg > 0;
                Pos nxt = p;
                WT Wn = W;
                if (more) {
                    const uint4 x = dev::philox4x32_10(
                        make_uint4(k, w, static_cast<uint32_t>(t), a.request), a.key0, a.key1);
                    nxt = step<WEIGHTED, WT>(g, p, x, a.scale, Wn);
                }
                wacc += static_cast<double>(static_cast<WT>(a.coef[t]) * W * static_cast<WT>(rl));
                if (DIGEST)
                    h = dev::fnv_step(h, p.l);
                ++nsteps;
                if (!more)
                    break;
                p = nxt;
                W = Wn;
                rl = r[p.l];
            }
            acc += wacc;
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
            q[k] = total / static_cast<double>(a.N);
            if (steps)
                atomicAdd(steps, st);
        }
    }
}

// Diagonal: visit records of start row kk, t-major: slot (kk*(K-1) + t)*N + w
// holds (l_t, c_{t+2} W_t); after a walk ends early its slots hold state -1.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF>
__global__ __launch_bounds__(256) void k_diag_walk(GraphView g, const int32_t *__restrict__ starts,
                                                   int64_t n_start, WalkArgs a,
                                                   int32_t *__restrict__ vstate,
                                                   WT *__restrict__ vx,
                                                   uint64_t *__restrict__ digest,
                                                   unsigned long long *steps) {
    __shared__ unsigned long long redu[4];
    const int last = a.K - 2;
    for (int64_t kk = blockIdx.x; kk < n_start; kk += gridDim.x) {
        const uint32_t k = static_cast<uint32_t>(starts[kk]);
        const uint2 rk = g.node[k];
        const int64_t row_base = kk * (a.K - 1) * a.N;
        uint64_t dig = 0;
        unsigned long long nsteps = 0;
        for (int64_t w64 = threadIdx.x; w64 < a.N; w64 += blockDim.x) {
            const uint32_t w = static_cast<uint32_t>(w64);
            Pos p{k, rk.x, rk.y};
            WT W = WT(1);
            uint64_t h = dev::kFnvBasis;
            int t = 0;
            for (; t <= last; ++t) {
                if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
                    break;
                const bool more = t < last && p.deg > 0;
                Pos nxt = p;
                WT Wn = W;
                if (more) {
                    const uint4 x = dev::philox4x32_10(
                        make_uint4(k, w, static_cast<uint32_t>(t), a.request), a.key0, a.key1);
                    nxt = step<WEIGHTED, WT>(g, p, x, a.scale, Wn);
                }
                const int64_t slot = row_base + int64_t(t) * a.N + w64;
                vstate[slot] = static_cast<int32_t>(p.l);
                vx[slot] = static_cast<WT>(a.coef[t]) * W;
                if (DIGEST)
                    h = dev::fnv_step(h, p.l);
                ++nsteps;
                if (!more) {
                    ++t;
                    break;
                }
                p = nxt;
                W = Wn;
            }
            for (; t <= last; ++t)
                vstate[row_base + int64_t(t) * a.N + w64] = -1;
            if (DIGEST)
                dig += h;
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

int walk_block(int64_t N) {
    if (N >= 256)
        return 256;
    return static_cast<int>(((N + 63) / 64) * 64);
}

// Workgroups loop over start rows, so the grid stays within the 32-bit
// work-item count of a dispatch whatever the number of start rows.
dim3 walk_grid(int64_t n_start) {
    const int64_t cap = int64_t(1) << 22;
    return dim3(static_cast<uint32_t>(n_start < cap ? n_start : cap));
}

// Runtime flags to template arguments.
template <class F>
void dispatch4(bool fp32, bool weighted, bool digest, bool cutoff, F &&f) {
    auto with_c = [&](auto wt, auto w, auto d) {
        if (cutoff)
            f(wt, w, d, std::true_type{});
        else
            f(wt, w, d, std::false_type{});
    };
    auto with_d = [&](auto wt, auto w) {
        if (digest)
            with_c(wt, w, std::true_type{});
        else
            with_c(wt, w, std::false_type{});
    };
    auto with_w = [&](auto wt) {
        if (weighted)
            with_d(wt, std::true_type{});
        else
            with_d(wt, std::false_type{});
    };
    if (fp32)
        with_w(float{});
    else
        with_w(double{});
}

} // namespace

Status action_walks(const mcmf_graph *g, const double *r, const int32_t *starts, int64_t n_start,
                    const WalkParams &p, double *q, uint64_t *digest, unsigned long long *steps,
                    hipStream_t s) {
    if (n_start <= 0 || p.K < 2)
        return {};
    const WalkArgs a = to_args(p);
    const GraphView gv = view(g);
    const dim3 grid = walk_grid(n_start), block(walk_block(p.n_walks));
    dispatch4(p.precision == MCMF_PRECISION_FP32_WEIGHTS, g->weighted, digest != nullptr,
              p.cutoff > 0.0, [&](auto wt, auto w, auto d, auto c) {
                  using WT = decltype(wt);
                  hipLaunchKernelGGL((k_action_walk<WT, decltype(w)::value, decltype(d)::value,
                                                    decltype(c)::value>),
                                     grid, block, 0, s, gv, r, starts, n_start, a, q, digest, steps);
              });
    MCMF_HIP(hipGetLastError());
    return {};
}

Status diag_walks(const mcmf_graph *g, const int32_t *starts, int64_t n_start, const WalkParams &p,
                  int32_t *state, void *x, uint64_t *digest, unsigned long long *steps,
                  hipStream_t s) {
    if (n_start <= 0 || p.K < 2)
        return {};
    const WalkArgs a = to_args(p);
    const GraphView gv = view(g);
    const dim3 grid = walk_grid(n_start), block(walk_block(p.n_walks));
    dispatch4(p.precision == MCMF_PRECISION_FP32_WEIGHTS, g->weighted, digest != nullptr,
              p.cutoff > 0.0, [&](auto wt, auto w, auto d, auto c) {
                  using WT = decltype(wt);
                  hipLaunchKernelGGL((k_diag_walk<WT, decltype(w)::value, decltype(d)::value,
                                                  decltype(c)::value>),
                                     grid, block, 0, s, gv, starts, n_start, a, state,
                                     static_cast<WT *>(x), digest, steps);
              });
    MCMF_HIP(hipGetLastError());
    return {};
}

} // namespace mcmf
