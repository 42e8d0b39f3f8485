// Device-side core of one random walk, shared by the single-request and
// the batched walk kernels.
//
// A walk keeps its state in registers: the current row l with its record
// (first entry, length) and the weight W.  A transition draws Philox4x32-10
// at counter (k, w, t, request), picks entry j of row l and moves to its
// column, multiplying W by s * sum_j |a_lj| (negated for a negative entry).
// Unweighted rows pick j = floor(u deg / 2^64) and read one 16-byte edge
// record {next row, its first entry, its length}: one dependent load per
// step.  The transition of step t is issued before step t is recorded, so
// the record's load overlaps the bookkeeping.  Weighted rows search the
// running sums of |a|.
//
// Weight type WT: double (FP64) or float (FP32 walk weights; W, the per-step
// factor and each per-step contribution are FP32, every sum stays FP64).
#pragma once

#include <type_traits>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {
namespace walk {

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
    const int32_t *row_walks; // null: N walks per start row
    const int64_t *row_rec;   // first visit record per start row (with row_walks)
    uint32_t hub_act;         // diag: hubs summed by the walk kernel (0: none)
    const uint8_t *in_set;    // diag: requested rows (null: all)
    double *dacc;             // diag: gather sums
};

inline WalkArgs to_args(const WalkParams &p) {
    WalkArgs a;
    a.coef = p.coef;
    a.K = p.K;
    a.scale = p.scale;
    a.N = p.n_walks;
    a.key0 = p.key0;
    a.key1 = p.key1;
    a.request = p.request;
    a.cutoff = p.cutoff;
    a.row_walks = p.row_walks;
    a.row_rec = p.row_rec;
    a.hub_act = p.hub_act;
    a.in_set = p.in_set;
    a.dacc = p.dacc;
    return a;
}

struct GraphView {
    const uint2 *node;
    const uint4 *edge;
    const int32_t *col;
    const double *val;
    const double *rowabs;
    const double *cum;
    const uint32_t *hubmask; // per node: adjacent hubs (null: no hubs)
    const int32_t *hub_row;  // hub index -> row
    const uint4 *alias;      // weighted rows: alias records (null: running sums)
};

// The graph's arrays for a walk launch; alias: weighted rows sample through
// the alias records (built by then).
inline GraphView view(const mcmf_graph *g, bool alias = false) {
    GraphView v;
    v.node = g->node;
    v.edge = g->edge;
    v.col = g->col;
    v.val = g->val;
    v.rowabs = g->rowabs;
    v.cum = g->cum;
    v.hubmask = g->hubmask;
    v.hub_row = g->hub_rows;
    v.alias = alias && g->weighted ? g->alias_rec : nullptr;
    return v;
}

// Walk state of one walk: row, its record and (EDGE records only) the mask
// of hubs adjacent to the row.
struct Pos {
    uint32_t l, start, deg, hm;
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Record loads; STREAM marks them non-temporal.  The entry a step picks is
// uniform over all stored entries (the walk's edge distribution), so records
// are rarely reused from cache; keeping them out of the cache can leave it to
// the vector the action walks read at every step (the autotuner decides).
template <bool STREAM>
__device__ __forceinline__ uint4 load_edge(const uint4 *e) {
    if constexpr (STREAM) {
        const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(e));
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *e;
    }
}

template <bool STREAM>
__device__ __forceinline__ int32_t load_col(const int32_t *c) {
    if constexpr (STREAM)
        return __builtin_nontemporal_load(c);
    else
        return *c;
}

// One transition out of row p (deg > 0) with the block of random words x.
// Updates W (times s * sum |a|, sign of the entry) and returns the new row.
// Unweighted rows either read one edge record (EDGE: the entry carries the
// next row's record) or the column and then the next row's record (two
// dependent loads, but 4 + 8 bytes instead of 16 and a row-record array
// that caches well); both pick the same entry.  Weighted rows search the
// running sums of |a|, or read one alias record (g.alias); the two map the
// random words to entries differently, with the same probabilities.
template <bool WEIGHTED, class WT, bool STREAM = false, bool EDGE = true>
__device__ __forceinline__ Pos step(const GraphView &g, const Pos &p, uint4 x, double scale,
                                    WT &W) {
    Pos n;
    if constexpr (!WEIGHTED) {
        const uint32_t j = dev::uniform_index(x.x, x.y, p.deg);
        W = W * static_cast<WT>(scale * static_cast<double>(p.deg));
        if constexpr (EDGE) {
            const uint4 e = load_edge<STREAM>(g.edge + (int64_t(p.start) + j));
            n.l = e.x;
            n.start = e.y;
            n.deg = e.z;
            n.hm = e.w;
        } else {
            n.l = static_cast<uint32_t>(load_col<STREAM>(g.col + (int64_t(p.start) + j)));
            const uint2 r = g.node[n.l];
            n.start = r.x;
            n.deg = r.y;
            n.hm = 0u;
        }
    } else if (g.alias) {
        // Alias method: entry i = floor(u deg / 2^64) from X0:X1, kept when
        // the 53-bit uniform from X2:X3 is below prob_i, else its alias.
        const double ra = g.rowabs[p.l];
        const uint32_t i = dev::uniform_index(x.x, x.y, p.deg);
        const uint4 r = g.alias[int64_t(p.start) + i];
        const double prob = __hiloint2double(static_cast<int>(r.w), static_cast<int>(r.z));
        const uint32_t c = dev::unit53(x.z, x.w) < prob ? r.x : r.y;
        W = W * static_cast<WT>(scale * ra);
        if (c >> 31)
            W = -W;
        n.l = c & 0x7fffffffu;
        const uint2 nr = g.node[n.l];
        n.start = nr.x;
        n.deg = nr.y;
        n.hm = 0u;
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
        n.hm = 0u;
    }
    return n;
}


// One action walk (walk index w from start row k): returns
// sum_t c_{t+2} W_t r_{l_t}; adds the recorded states to *nsteps and folds
// the path into *h.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF, bool EDGE = true, bool STREAM = true>
__device__ __forceinline__ double action_walk(const GraphView &g, const double *__restrict__ r,
                                              const WalkArgs &a, uint32_t k, uint2 rk, double r_k,
                                              uint32_t w, uint64_t *h, unsigned long long *nsteps) {
    const int last = a.K - 2;
    Pos p{k, rk.x, rk.y, 0u};
    double rl = r_k;
    WT W = WT(1);
    double wacc = 0.0;
    for (int t = 0; t <= last; ++t) {
        if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
            break;
        const bool more = t < last && p.deg > 0;
        Pos nxt = p;
        WT Wn = W;
        if (more) {
            const uint4 x = dev::philox4x32_10(make_uint4(k, w, static_cast<uint32_t>(t), a.request),
                                               a.key0, a.key1);
            nxt = step<WEIGHTED, WT, STREAM, EDGE>(g, p, x, a.scale, Wn);
        }
        wacc += static_cast<double>(static_cast<WT>(a.coef[t]) * W * static_cast<WT>(rl));
        if (DIGEST)
            *h = dev::fnv_step(*h, p.l);
        ++*nsteps;
        if (!more)
            break;
        p = nxt;
        W = Wn;
        rl = r[p.l];
    }
    return wacc;
}

// One action walk over value records (unweighted rows): rec[e] = {first
// entry of row col[e], its length, r[col[e]] as two words}, built per call,
// so a step loads one 16-byte record and needs no separate read of r.  The
// walk is the same as action_walk's (same draws, entries, weights and sum);
// only the row index itself is not carried.
template <class WT, bool CUTOFF, bool STREAM>
__device__ __forceinline__ double action_walk_value(const uint4 *__restrict__ rec, const WalkArgs &a,
                                                    uint32_t k, uint2 rk, double r_k, uint32_t w,
                                                    unsigned long long *nsteps) {
    const int last = a.K - 2;
    uint32_t start = rk.x, deg = rk.y;
    double rl = r_k;
    WT W = WT(1);
    double wacc = 0.0;
    for (int t = 0; t <= last; ++t) {
        if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
            break;
        const bool more = t < last && deg > 0;
        uint32_t n_start = start, n_deg = deg;
        double n_r = rl;
        WT Wn = W;
        if (more) {
            const uint4 x = dev::philox4x32_10(make_uint4(k, w, static_cast<uint32_t>(t), a.request),
                                               a.key0, a.key1);
            const uint32_t j = dev::uniform_index(x.x, x.y, deg);
            Wn = W * static_cast<WT>(a.scale * static_cast<double>(deg));
            const uint4 e = load_edge<STREAM>(rec + (int64_t(start) + j));
            n_start = e.x;
            n_deg = e.y;
            n_r = __hiloint2double(static_cast<int>(e.w), static_cast<int>(e.z));
        }
        wacc += static_cast<double>(static_cast<WT>(a.coef[t]) * W * static_cast<WT>(rl));
        ++*nsteps;
        if (!more)
            break;
        start = n_start;
        deg = n_deg;
        W = Wn;
        rl = n_r;
    }
    return wacc;
}

// One diagonal walk: writes (l_t, c_{t+2} W_t) to vstate[t*stride],
// vx[t*stride] for t = 0..K-2 (state -1 once the walk has ended).  With
// hub_k != 0 (unweighted graphs; the hubs adjacent to k whose sums this
// walk feeds) each recorded weight is also added to hsum[h] (LDS) for every
// hub h in hub_k adjacent to l_t: the walk's share of <Q_k, C_h>.
template <class WT, bool WEIGHTED, bool DIGEST, bool CUTOFF, bool EDGE = true, bool STREAM = false>
__device__ __forceinline__ void diag_walk(const GraphView &g, const WalkArgs &a, uint32_t k,
                                          uint2 rk, uint32_t w, int32_t *__restrict__ vstate,
                                          WT *__restrict__ vx, int64_t stride, uint64_t *h,
                                          unsigned long long *nsteps, uint32_t hub_k = 0u,
                                          double *hsum = nullptr) {
    const int last = a.K - 2;
    // k itself is adjacent to every hub in hub_k.
    Pos p{k, rk.x, rk.y, hub_k};
    WT W = WT(1);
    int t = 0;
    for (; t <= last; ++t) {
        if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
            break;
        const bool more = t < last && p.deg > 0;
        Pos nxt = p;
        WT Wn = W;
        if (more) {
            const uint4 x = dev::philox4x32_10(make_uint4(k, w, static_cast<uint32_t>(t), a.request),
                                               a.key0, a.key1);
            nxt = step<WEIGHTED, WT, STREAM, EDGE>(g, p, x, a.scale, Wn);
        }
        const WT xt = static_cast<WT>(a.coef[t]) * W;
        vstate[int64_t(t) * stride] = static_cast<int32_t>(p.l);
        vx[int64_t(t) * stride] = xt;
        if constexpr (!WEIGHTED) {
            if (hub_k != 0u) {
                uint32_t m = ((EDGE || t == 0) ? p.hm : g.hubmask[p.l]) & hub_k;
                while (m != 0u) {
                    atomicAdd(&hsum[__ffs(m) - 1], static_cast<double>(xt));
                    m &= m - 1u;
                }
            }
        }
        if (DIGEST)
            *h = dev::fnv_step(*h, p.l);
        ++*nsteps;
        if (!more) {
            ++t;
            break;
        }
        p = nxt;
        W = Wn;
    }
    for (; t <= last; ++t)
        vstate[int64_t(t) * stride] = -1;
}

// Requested wide hubs adjacent to a start row k (uniform over the row's
// walks): mask word w of them, and the 16-byte chunks of a node's 128-byte
// wide mask that hold the nonzero words.
struct WideRow {
    uint32_t hk[kWideWords];
    uint32_t chunks; // bit c: words 4c..4c+3 are needed
    bool any;
};

// Word i (0..3) of a uint4, i known at compile time after unrolling.
__device__ __forceinline__ uint32_t word_of(const uint4 &v, int i) {
    return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// One diagonal walk over edge records with wide hub sums (unweighted
// graphs): the visit records as diag_walk writes them, and for every visit
// (t >= 1) at a state l adjacent to one of the hubs in hr its weight added to
// hsum[h] (LDS).  The needed chunks of l's wide mask are loaded together with
// the record of the step out of l, so their latency hides behind it.  Step 0
// sits at k, adjacent to every hub in hr: its weights go to *acc0, added to
// every such hub once per start row.
template <class WT, bool DIGEST, bool CUTOFF>
__device__ __forceinline__ void diag_walk_wide(const uint4 *__restrict__ edge, const uint4 *__restrict__ wmask,
                                               const WalkArgs &a, uint32_t k, uint2 rk, uint32_t w,
                                               int32_t *__restrict__ vstate, WT *__restrict__ vx, int64_t stride,
                                               uint64_t *h, unsigned long long *nsteps, const WideRow &hr,
                                               double *hsum, double *acc0) {
    const int last = a.K - 2;
    uint32_t l = k, start = rk.x, deg = rk.y;
    WT W = WT(1);
    int t = 0;
    for (; t <= last; ++t) {
        if (CUTOFF && !(fabs(static_cast<double>(W)) > a.cutoff))
            break;
        const bool more = t < last && deg > 0;
        const bool sums = hr.any && t > 0;
        uint4 c[kWideWords / 4];
        if (sums) {
            const uint4 *ml = wmask + int64_t(l) * (kWideWords / 4);
#pragma unroll
            for (int q = 0; q < kWideWords / 4; ++q)
                if ((hr.chunks >> q) & 1u)
                    c[q] = ml[q];
        }
        uint4 nx = make_uint4(l, start, deg, 0u);
        WT Wn = W;
        if (more) {
            const uint4 x = dev::philox4x32_10(make_uint4(k, w, static_cast<uint32_t>(t), a.request),
                                               a.key0, a.key1);
            const uint32_t j = dev::uniform_index(x.x, x.y, deg);
            Wn = W * static_cast<WT>(a.scale * static_cast<double>(deg));
            nx = edge[int64_t(start) + j];
        }
        const WT xt = static_cast<WT>(a.coef[t]) * W;
        vstate[int64_t(t) * stride] = static_cast<int32_t>(l);
        vx[int64_t(t) * stride] = xt;
        if (t == 0 && hr.any)
            *acc0 += static_cast<double>(xt);
        if (sums) {
#pragma unroll
            for (int wd = 0; wd < kWideWords; ++wd) {
                if (hr.hk[wd] == 0u)
                    continue;
                uint32_t m = word_of(c[wd >> 2], wd & 3) & hr.hk[wd];
                while (m != 0u) {
                    atomicAdd(&hsum[32 * wd + __ffs(m) - 1], static_cast<double>(xt));
                    m &= m - 1u;
                }
            }
        }
        if (DIGEST)
            *h = dev::fnv_step(*h, l);
        ++*nsteps;
        if (!more) {
            ++t;
            break;
        }
        l = nx.x;
        start = nx.y;
        deg = nx.z;
        W = Wn;
    }
    for (; t <= last; ++t)
        vstate[int64_t(t) * stride] = -1;
}

// Runtime flags to template arguments, sampler layout included (weighted
// rows have one layout: the sampler flags are ignored for them).
template <class F>
void dispatch6(bool fp32, bool weighted, bool digest, bool cutoff, bool edge, bool stream, F &&f) {
    auto with_s = [&](auto wt, auto w, auto d, auto c, auto e) {
        if (stream && !decltype(w)::value)
            f(wt, w, d, c, e, std::true_type{});
        else
            f(wt, w, d, c, e, std::false_type{});
    };
    auto with_e = [&](auto wt, auto w, auto d, auto c) {
        if (edge || decltype(w)::value)
            with_s(wt, w, d, c, std::true_type{});
        else
            with_s(wt, w, d, c, std::false_type{});
    };
    auto with_c = [&](auto wt, auto w, auto d) {
        if (cutoff)
            with_e(wt, w, d, std::true_type{});
        else
            with_e(wt, w, d, std::false_type{});
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

} // namespace walk
} // namespace mcmf
