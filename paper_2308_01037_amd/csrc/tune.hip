// Autotuner of the walk kernels (mcmf_tune) and the tuning accessors.
//
// The walk step has two sampler layouts (one 16-byte edge record, or the
// column and then the next row's record) and two load policies (cached or
// non-temporal); the action walk of an unweighted graph has a third layout,
// per-call value records that carry r of the next row.  Which is fastest
// depends on the graph: its size against the caches, the locality of its
// node numbering, the degree spread.  The tuner times every variant of the
// action walk (value records included, their build counted) and of the
// diagonal walk on an evenly strided sample of the rows with entries, with
// the caller's function, walk count and K, and keeps the fastest of each.
#include <algorithm>
#include <cmath>
#include <vector>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

__global__ void k_stride_sample(const int32_t *__restrict__ active, int64_t stride, int64_t m,
                                int32_t *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m)
        out[i] = active[i * stride];
}

Status check_tuning(const mcmf_tuning *t) {
    if (!t)
        return fail(MCMF_E_ARG, "tuning is NULL");
    auto sampler_ok = [](int32_t v) { return v == MCMF_SAMPLER_EDGE || v == MCMF_SAMPLER_ROW; };
    auto flag_ok = [](int32_t v) { return v == 0 || v == 1; };
    if (!(sampler_ok(t->action_sampler) || t->action_sampler == MCMF_SAMPLER_VALUE) ||
        !sampler_ok(t->diag_sampler))
        return fail(MCMF_E_ARG, "unknown sampler layout (VALUE is for the action only)");
    if (!flag_ok(t->action_stream) || !flag_ok(t->diag_stream))
        return fail(MCMF_E_ARG, "stream flags must be 0 or 1");
    if (t->hub_min_degree < 0)
        return fail(MCMF_E_ARG, "hub_min_degree must be >= 0 (got %d)", t->hub_min_degree);
    return {};
}

Status tune(mcmf_graph *g, const mcmf_fn *f, int64_t N, int32_t K, mcmf_tuning *out) {
    MCMF_TRY(check_common(g, f, N, K, nullptr));
    if (!out)
        return fail(MCMF_E_ARG, "out is NULL");
    if (K < 2)
        return fail(MCMF_E_ARG, "mcmf_tune needs K >= 2 (K = %d)", K);
    MCMF_HIP(hipSetDevice(g->device));
    hipStream_t s = g->stream;
    mcmf_tuning best = g->tuning;
    best.sample_rows = 0;
    for (double &x : best.action_ms)
        x = 0.0;
    for (double &x : best.diag_ms)
        x = 0.0;
    for (double &x : best.action_value_ms)
        x = 0.0;
    if (g->n_active == 0) {
        *out = best;
        return {};
    }
    // Sample: about 2^28 walk steps, and at most 512 MiB of visit records.
    const int64_t per_row = N * (K - 1);
    int64_t m = std::max<int64_t>(1, (int64_t(1) << 28) / per_row);
    m = std::min<int64_t>(m, std::max<int64_t>(1, (int64_t(512) << 20) / (per_row * 12)));
    m = std::min<int64_t>(m, g->n_active);
    const int64_t stride = g->n_active / m;
    DevBuf<int32_t> rows;
    MCMF_TRY(rows.alloc(m, s));
    hipLaunchKernelGGL(k_stride_sample, dim3(static_cast<uint32_t>((m + 255) / 256)), dim3(256), 0, s,
                       g->active, stride, m, rows.ptr);
    MCMF_HIP(hipGetLastError());
    std::vector<double> c(K + 1);
    MCMF_TRY(make_coeffs(f, K, c.data()));
    DevBuf<double> coef, ones, r, q;
    DevBuf<int32_t> vstate;
    DevBuf<double> vx;
    DevBuf<unsigned long long> steps;
    const int64_t n = g->n;
    MCMF_TRY(coef.alloc(K - 1, s));
    MCMF_HIP(hipMemcpyAsync(coef.ptr, c.data() + 2, sizeof(double) * (K - 1), hipMemcpyHostToDevice, s));
    MCMF_TRY(ones.alloc(n, s));
    MCMF_TRY(r.alloc(n, s));
    MCMF_TRY(q.alloc(n, s));
    MCMF_TRY(vstate.alloc(m * per_row, s));
    MCMF_TRY(vx.alloc(m * per_row, s));
    MCMF_TRY(steps.alloc(1, s));
    MCMF_TRY(fill_f64(ones.ptr, 1.0, n, s));
    MCMF_TRY(spmv_r(g, ones.ptr, f->scale, r.ptr, s));
    WalkParams p = walk_params(nullptr, coef.ptr, K, f->scale, N);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    MCMF_HIP(hipEventCreate(&e0));
    MCMF_HIP(hipEventCreate(&e1));
    struct Events {
        hipEvent_t a, b;
        ~Events() {
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
        }
    } guard{e0, e1};
    // Best of three timed launches after one warm-up.
    auto time_it = [&](auto &&launch, double *ms) -> Status {
        MCMF_TRY(launch());
        double bestms = 1e300;
        for (int rep = 0; rep < 3; ++rep) {
            MCMF_HIP(hipEventRecord(e0, s));
            MCMF_TRY(launch());
            MCMF_HIP(hipEventRecord(e1, s));
            MCMF_HIP(hipEventSynchronize(e1));
            float t = 0.f;
            MCMF_HIP(hipEventElapsedTime(&t, e0, e1));
            bestms = std::min(bestms, static_cast<double>(t));
        }
        *ms = bestms;
        return {};
    };
    for (int v = 0; v < 4; ++v) {
        p.sampler = v >> 1;
        p.stream = v & 1;
        MCMF_TRY(time_it([&]() { return action_walks(g, r.ptr, rows.ptr, m, p, q.ptr, nullptr, steps.ptr, s); },
                         &best.action_ms[v]));
        MCMF_TRY(time_it([&]() {
            return diag_walks(g, rows.ptr, m, p, vstate.ptr, vx.ptr, nullptr, steps.ptr, s);
        }, &best.diag_ms[v]));
    }
    int ba = 0, bd = 0;
    for (int v = 1; v < 4; ++v) {
        if (best.action_ms[v] < best.action_ms[ba])
            ba = v;
        if (best.diag_ms[v] < best.diag_ms[bd])
            bd = v;
    }
    // Weighted graphs have one layout: the choice only matters unweighted.
    best.action_sampler = ba >> 1;
    best.action_stream = ba & 1;
    // Value records (unweighted graphs that can hold them); the record build
    // is part of the timed call.
    if (!g->weighted && value_records_fit(g)) {
        for (int st = 0; st < 2; ++st) {
            p.sampler = MCMF_SAMPLER_VALUE;
            p.stream = st;
            MCMF_TRY(time_it([&]() { return action_walks(g, r.ptr, rows.ptr, m, p, q.ptr, nullptr, steps.ptr, s); },
                             &best.action_value_ms[st]));
        }
        const int st = best.action_value_ms[0] <= best.action_value_ms[1] ? 0 : 1;
        if (best.action_value_ms[st] < best.action_ms[ba]) {
            best.action_sampler = MCMF_SAMPLER_VALUE;
            best.action_stream = st;
        }
    }
    best.diag_sampler = bd >> 1;
    best.diag_stream = bd & 1;
    best.sample_rows = m;
    MCMF_HIP(hipStreamSynchronize(s));
    g->tuning = best;
    *out = best;
    out->hub_count = g->n_hubs;
    return {};
}

} // namespace

} // namespace mcmf

extern "C" mcmf_status mcmf_graph_set_tuning(mcmf_graph *g, const mcmf_tuning *t) {
    mcmf::clear_error();
    if (!g) {
        mcmf::fail(MCMF_E_ARG, "graph is NULL");
        return MCMF_E_ARG;
    }
    mcmf::Status st = mcmf::check_tuning(t);
    if (st)
        return st.code;
    g->tuning.action_sampler = t->action_sampler;
    g->tuning.action_stream = t->action_stream;
    g->tuning.diag_sampler = t->diag_sampler;
    g->tuning.diag_stream = t->diag_stream;
    g->tuning.hub_min_degree = t->hub_min_degree;
    return MCMF_OK;
}

extern "C" mcmf_status mcmf_graph_get_tuning(const mcmf_graph *g, mcmf_tuning *t) {
    mcmf::clear_error();
    if (!g || !t) {
        mcmf::fail(MCMF_E_ARG, "graph and tuning must not be NULL");
        return MCMF_E_ARG;
    }
    *t = g->tuning;
    t->hub_count = g->n_hubs;
    return MCMF_OK;
}

extern "C" mcmf_status mcmf_tune(mcmf_graph *g, const mcmf_fn *f, int64_t n_walks, int32_t K,
                                 mcmf_tuning *out) {
    mcmf::clear_error();
    return mcmf::tune(g, f, n_walks, K, out).code;
}
