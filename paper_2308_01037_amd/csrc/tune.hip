// Autotuner of the walk and gather kernels (mcmf_tune) and the tuning
// accessors.
//
// The walk step has two sampler layouts (one 16-byte edge record, or the
// column and then the next row's record) and two load policies (cached or
// non-temporal); the action walk of an unweighted graph has a third layout,
// per-call value records that carry r of the next row.  A start row's walks
// run on 64, 128 or 256 lanes.  The diagonal gather cuts a start row's
// neighbours into work items (each rebuilds Q_k) and may leave the graph's
// hub rows to sums taken by the walk.  Which choices are fastest depends on
// the graph: its size against the caches, the locality of its node
// numbering, the degree spread.  The tuner times the variants of each stage
// on an evenly strided sample of the rows with entries, with the caller's
// function, walk count and K, and keeps the fastest of each.
#include <algorithm>
#include <climits>
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
    if (!(sampler_ok(t->action_sampler) || t->action_sampler == MCMF_SAMPLER_VALUE ||
          t->action_sampler == MCMF_SAMPLER_ALIAS) ||
        !(sampler_ok(t->diag_sampler) || t->diag_sampler == MCMF_SAMPLER_WIDE || t->diag_sampler == MCMF_SAMPLER_ALIAS ||
          t->diag_sampler == MCMF_SAMPLER_AUTO))
        return fail(MCMF_E_ARG, "unknown sampler layout (VALUE is for the action only, WIDE and AUTO for the diagonal)");
    if (!flag_ok(t->action_stream) || !flag_ok(t->diag_stream))
        return fail(MCMF_E_ARG, "stream flags must be 0 or 1");
    if (t->hub_min_degree < 0)
        return fail(MCMF_E_ARG, "hub_min_degree must be >= 0 (got %d)", t->hub_min_degree);
    if (t->walk_threads != 0 && t->walk_threads != 64 && t->walk_threads != 128 && t->walk_threads != 256)
        return fail(MCMF_E_ARG, "walk_threads must be 0, 64, 128 or 256 (got %d)", t->walk_threads);
    if (t->gather_item != 0 && (t->gather_item < 64 || t->gather_item > 4096))
        return fail(MCMF_E_ARG, "gather_item must be 0 or within [64, 4096] (got %d)", t->gather_item);
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
    for (double &x : best.walk_threads_ms)
        x = 0.0;
    for (double &x : best.gather_item_ms)
        x = 0.0;
    for (double &x : best.hub_ms)
        x = 0.0;
    best.wide_ms = 0.0;
    best.alias_ms[0] = best.alias_ms[1] = 0.0;
    if (g->n_active == 0) {
        *out = best;
        return {};
    }
    // Sample: about 2^28 walk steps, and at most 2 GiB (or 1/32 of device
    // memory) of visit records: the gather's launches need enough work items
    // per workgroup for their tails to weigh as little as in a full query.
    const int64_t per_row = N * (K - 1);
    const int64_t visit_cap = std::min<int64_t>(int64_t(2) << 30, static_cast<int64_t>(device_memory_bytes() / 32));
    int64_t m = std::max<int64_t>(1, (int64_t(1) << 28) / per_row);
    m = std::min<int64_t>(m, std::max<int64_t>(1, visit_cap / (per_row * 12)));
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
    // Value records (unweighted graphs that can hold them).  A call builds
    // them once for the whole graph, so the build is charged in proportion
    // to the sample's share of the start rows, as a full query would carry it.
    if (!g->weighted && value_records_fit(g)) {
        double build_ms = 0.0;
        {
            DevBuf<uint4> rec;
            MCMF_TRY(rec.alloc(g->nnz, s));
            MCMF_TRY(time_it([&]() { return build_value_records(g, r.ptr, rec.ptr, s); }, &build_ms));
        }
        const double share = static_cast<double>(m) / static_cast<double>(g->n_active);
        for (int st = 0; st < 2; ++st) {
            p.sampler = MCMF_SAMPLER_VALUE;
            p.stream = st;
            double ms = 0.0;
            MCMF_TRY(time_it([&]() { return action_walks(g, r.ptr, rows.ptr, m, p, q.ptr, nullptr, steps.ptr, s); },
                             &ms));
            best.action_value_ms[st] = std::max(0.0, ms - build_ms) + build_ms * share;
        }
        const int st = best.action_value_ms[0] <= best.action_value_ms[1] ? 0 : 1;
        if (best.action_value_ms[st] < best.action_ms[ba]) {
            best.action_sampler = MCMF_SAMPLER_VALUE;
            best.action_stream = st;
        }
    }
    best.diag_sampler = bd >> 1;
    best.diag_stream = bd & 1;
    // Weighted graphs: the running sums (any of the four above) against the
    // alias records (unless those do not fit).
    Status alias_room = g->weighted ? ensure_alias(g) : Status{};
    if (alias_room && alias_room.code != MCMF_E_NOMEM)
        return alias_room;
    if (alias_room)
        clear_error();
    if (g->weighted && !alias_room) {
        p.sampler = MCMF_SAMPLER_ALIAS;
        p.stream = 0;
        MCMF_TRY(time_it([&]() { return action_walks(g, r.ptr, rows.ptr, m, p, q.ptr, nullptr, steps.ptr, s); },
                         &best.alias_ms[0]));
        MCMF_TRY(time_it([&]() {
            return diag_walks(g, rows.ptr, m, p, vstate.ptr, vx.ptr, nullptr, steps.ptr, s);
        }, &best.alias_ms[1]));
        if (best.alias_ms[0] < best.action_ms[ba]) {
            best.action_sampler = MCMF_SAMPLER_ALIAS;
            best.action_stream = 0;
        }
        if (best.alias_ms[1] < best.diag_ms[bd]) {
            best.diag_sampler = MCMF_SAMPLER_ALIAS;
            best.diag_stream = 0;
        }
    }
    p.sampler = best.diag_sampler;
    p.stream = best.diag_stream;

    // Lanes per start row of the walks (timed on the diagonal walk).
    const int lanes[3] = {64, 128, 256};
    for (int i = 0; i < 3; ++i) {
        p.threads = lanes[i];
        MCMF_TRY(time_it([&]() {
            return diag_walks(g, rows.ptr, m, p, vstate.ptr, vx.ptr, nullptr, steps.ptr, s);
        }, &best.walk_threads_ms[i]));
    }
    // Another choice than the default must win by more than kMargin: the
    // sample's timings carry noise of a few per cent.
    constexpr double kMargin = 0.97;
    int bt = 2;
    for (int i = 1; i >= 0; --i)
        if (best.walk_threads_ms[i] < kMargin * best.walk_threads_ms[bt])
            bt = i;
    best.walk_threads = lanes[bt];
    p.threads = lanes[bt];

    // The diagonal gather over the sample (every neighbour of a sampled row
    // requested): work-item size, then hub sums on and off.
    if (g->symmetric) {
        DevBuf<double> dacc;
        DevBuf<int64_t> items;
        DevBuf<unsigned long long> counters; // probes, overflow, queue
        MCMF_TRY(dacc.alloc(n, s));
        MCMF_TRY(items.alloc(m + 1, s));
        MCMF_TRY(counters.alloc(3, s));
        const uint32_t auto_hubs = g->weighted ? 0u : active_hubs(g, N, K);
        auto run_diag = [&](uint32_t item, uint32_t hubs, bool walk, int32_t whubs = -1) -> Status {
            WalkParams pd = p;
            pd.gather_item = item;
            pd.hub_act = hubs;
            if (whubs >= 0) {
                pd.sampler = MCMF_SAMPLER_WIDE;
                pd.whub_act = whubs;
                pd.hub_act = 0u;
            }
            pd.in_set = nullptr;
            pd.dacc = dacc.ptr;
            MCMF_TRY(fill_f64(dacc.ptr, 0.0, n, s));
            MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(counters.ptr), 0, 3, s));
            if (walk)
                MCMF_TRY(diag_walks(g, rows.ptr, m, pd, vstate.ptr, vx.ptr, nullptr, steps.ptr, s));
            return diag_gather(g, rows.ptr, items.ptr, 0, m, pd, vstate.ptr, vx.ptr, nullptr, dacc.ptr,
                               counters.ptr, counters.ptr + 1, counters.ptr + 2, s);
        };
        const uint32_t sizes[4] = {128, 256, 512, 1024};
        MCMF_TRY(gather_items(g, rows.ptr, m, items.ptr, s, sizes[1]));
        MCMF_TRY(run_diag(sizes[1], auto_hubs, true)); // visit records of the sample
        for (int i = 0; i < 4; ++i) {
            MCMF_TRY(gather_items(g, rows.ptr, m, items.ptr, s, sizes[i]));
            MCMF_TRY(time_it([&]() { return run_diag(sizes[i], auto_hubs, false); }, &best.gather_item_ms[i]));
        }
        int bi = 1; // the default unless another size wins by the margin
        for (int i = 0; i < 4; ++i)
            if (i != 1 && best.gather_item_ms[i] < kMargin * best.gather_item_ms[1] &&
                best.gather_item_ms[i] < best.gather_item_ms[bi])
                bi = i;
        best.gather_item = static_cast<int32_t>(sizes[bi]);
        MCMF_TRY(gather_items(g, rows.ptr, m, items.ptr, s, sizes[bi]));
        if (auto_hubs != 0u) {
            MCMF_TRY(time_it([&]() { return run_diag(sizes[bi], auto_hubs, true); }, &best.hub_ms[0]));
            MCMF_TRY(time_it([&]() { return run_diag(sizes[bi], 0u, true); }, &best.hub_ms[1]));
            best.hub_min_degree = best.hub_ms[1] < kMargin * best.hub_ms[0] ? INT32_MAX : 0;
        }
        // Wide hubs: walk and gather with the wide hub sums at the automatic
        // threshold, against the better of the two above.  The graph's
        // current layout stays unless the other wins by the margin.
        if (g->n_whubs > 0 && !g->weighted) {
            const int32_t wide_act = active_wide_hubs(g, N, K);
            MCMF_TRY(time_it([&]() { return run_diag(sizes[bi], 0u, true, wide_act); }, &best.wide_ms));
            double other = std::min(best.hub_ms[0], best.hub_ms[1]);
            if (auto_hubs == 0u)
                MCMF_TRY(time_it([&]() { return run_diag(sizes[bi], 0u, true); }, &other));
            const bool wide_now = g->tuning.diag_sampler == MCMF_SAMPLER_WIDE ||
                                  (g->tuning.diag_sampler == MCMF_SAMPLER_AUTO && auto_wide(g, N, K));
            if (wide_now ? !(other < kMargin * best.wide_ms) : best.wide_ms < kMargin * other) {
                best.diag_sampler = MCMF_SAMPLER_WIDE;
                best.diag_stream = 0;
                best.hub_min_degree = 0;
            }
        }
        unsigned long long lost = 0;
        MCMF_HIP(hipMemcpyAsync(&lost, counters.ptr + 1, sizeof lost, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipStreamSynchronize(s));
        if (lost != 0)
            return fail(MCMF_E_DEVICE, "internal error: a Q_k table overflowed while tuning");
    }
    best.sample_rows = m;
    MCMF_HIP(hipStreamSynchronize(s));
    const bool items_changed = best.gather_item != g->tuning.gather_item;
    g->tuning = best;
    if (items_changed)
        MCMF_TRY(refresh_active_items(g));
    *out = best;
    out->hub_count = g->n_hubs;
    out->wide_hub_count = g->n_whubs;
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
    if (t->diag_sampler == MCMF_SAMPLER_WIDE && g->n_whubs == 0) {
        mcmf::fail(MCMF_E_ARG, "diag_sampler WIDE needs a graph with wide hubs");
        return MCMF_E_ARG;
    }
    if ((t->action_sampler == MCMF_SAMPLER_ALIAS || t->diag_sampler == MCMF_SAMPLER_ALIAS) && !g->weighted) {
        mcmf::fail(MCMF_E_ARG, "the ALIAS sampler is for weighted graphs");
        return MCMF_E_ARG;
    }
    if (t->action_sampler == MCMF_SAMPLER_ALIAS || t->diag_sampler == MCMF_SAMPLER_ALIAS) {
        st = mcmf::ensure_alias(g);
        if (st)
            return st.code;
    }
    g->tuning.action_sampler = t->action_sampler;
    g->tuning.action_stream = t->action_stream;
    g->tuning.diag_sampler = t->diag_sampler;
    g->tuning.diag_stream = t->diag_stream;
    g->tuning.hub_min_degree = t->hub_min_degree;
    g->tuning.walk_threads = t->walk_threads;
    if (t->gather_item != g->tuning.gather_item) {
        g->tuning.gather_item = t->gather_item;
        st = mcmf::refresh_active_items(g);
        if (st)
            return st.code;
    }
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
    t->wide_hub_count = g->n_whubs;
    return MCMF_OK;
}

extern "C" mcmf_status mcmf_tune(mcmf_graph *g, const mcmf_fn *f, int64_t n_walks, int32_t K,
                                 mcmf_tuning *out) {
    mcmf::clear_error();
    return mcmf::tune(g, f, n_walks, K, out).code;
}
