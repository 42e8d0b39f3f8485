// Entry points mcmf_action and mcmf_diag: argument checks, marshalling of
// host/device buffers, the start set, chunking of the diagonal's visit
// buffer, statistics, and the small kernels that assemble the diagonal.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

constexpr int kMaxK = 4096;

// ---- small kernels ----

// in_set[i] = 1 for every requested row; counts rows outside [0, n).
__global__ void k_mark_rows(const int32_t *rows, int64_t n_rows, int64_t n, uint8_t *in_set,
                            int *bad) {
    for (int64_t p = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; p < n_rows;
         p += int64_t(gridDim.x) * blockDim.x) {
        const int32_t i = rows[p];
        if (i < 0 || i >= n)
            atomicOr(bad, 1);
        else
            in_set[i] = 1;
    }
}

// start[k] = 1 for every k adjacent to a requested row (one wavefront per row).
__global__ __launch_bounds__(256) void k_mark_starts(const int32_t *rows, int64_t n_rows,
                                                     const uint2 *node, const int32_t *col,
                                                     uint8_t *start) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / 64);
    for (int64_t p = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6); p < n_rows;
         p += waves) {
        const uint2 ri = node[rows[p]];
        for (uint32_t e = lane; e < ri.y; e += 64)
            start[col[int64_t(ri.x) + e]] = 1;
    }
}

// out[p] = c0 + c1 s a_ii + dacc[i], i = rows[p] (rows null: i = p).
// a_ii is the sum of the stored (i, i) entries (one wavefront per output).
__global__ __launch_bounds__(256) void k_diag_finish(const int32_t *rows, int64_t count,
                                                     const uint2 *node, const int32_t *col,
                                                     const double *val, int K, double c0, double c1,
                                                     double scale, const double *dacc,
                                                     double *out) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / 64);
    for (int64_t p = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6); p < count;
         p += waves) {
        const int32_t i = rows ? rows[p] : static_cast<int32_t>(p);
        double aii = 0.0;
        if (K >= 1) {
            const uint2 ri = node[i];
            for (uint32_t e = lane; e < ri.y; e += 64) {
                const int64_t idx = int64_t(ri.x) + e;
                if (col[idx] == i)
                    aii += val ? val[idx] : 1.0;
            }
            aii = dev::wave_sum(aii);
        }
        if (lane == 0) {
            double d = c0;
            if (K >= 1)
                d = d + c1 * (scale * aii);
            if (K >= 2)
                d = d + dacc[i];
            out[p] = d;
        }
    }
}

int64_t grid_for(int64_t n, int per_block) {
    int64_t b = (n + per_block - 1) / per_block;
    const int64_t cap = int64_t(1) << 20;
    return b < 1 ? 1 : (b < cap ? b : cap);
}

} // namespace

Status mark_rows(const int32_t *rows, int64_t count, int64_t n, uint8_t *in_set, int *bad,
                 hipStream_t s) {
    if (count <= 0)
        return {};
    hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(count, 256)), dim3(256), 0, s, rows, count, n,
                       in_set, bad);
    MCMF_HIP(hipGetLastError());
    return {};
}

Status mark_starts(const mcmf_graph *g, const int32_t *rows, int64_t count, uint8_t *start_flags,
                   hipStream_t s) {
    if (count <= 0)
        return {};
    hipLaunchKernelGGL(k_mark_starts, dim3(grid_for(count, 4)), dim3(256), 0, s, rows, count,
                       g->node, g->col, start_flags);
    MCMF_HIP(hipGetLastError());
    return {};
}

Status diag_finish(const mcmf_graph *g, const int32_t *rows, int64_t count, int K, double c0,
                   double c1, double scale, const double *dacc, double *out, hipStream_t s) {
    if (count <= 0)
        return {};
    hipLaunchKernelGGL(k_diag_finish, dim3(grid_for(count, 4)), dim3(256), 0, s, rows, count,
                       g->node, g->col, g->val, K, c0, c1, scale, dacc, out);
    MCMF_HIP(hipGetLastError());
    return {};
}

namespace {

// ---- argument handling ----

} // namespace

WalkParams walk_params(const mcmf_opts *o, const double *coef, int K, double scale, int64_t N) {
    WalkParams p;
    p.coef = coef;
    p.K = K;
    p.scale = scale;
    p.n_walks = N;
    const uint64_t seed = o ? o->seed : 0;
    p.key0 = static_cast<uint32_t>(seed & 0xffffffffu);
    p.key1 = static_cast<uint32_t>(seed >> 32);
    p.request = o ? o->request_id : 0u;
    p.cutoff = o ? o->weight_cutoff : 0.0;
    p.precision = o ? o->precision : 0;
    return p;
}

Status check_common(const mcmf_graph *g, const mcmf_fn *f, int64_t n_walks, int32_t K,
                    const mcmf_opts *o) {
    if (!g)
        return fail(MCMF_E_ARG, "graph is NULL");
    if (!f)
        return fail(MCMF_E_ARG, "function is NULL");
    if (K < 0 || K > kMaxK)
        return fail(MCMF_E_ARG, "K = %d outside [0, %d]", K, kMaxK);
    if (K >= 2 && (n_walks < 1 || n_walks > (int64_t(1) << 32)))
        return fail(MCMF_E_ARG, "n_walks = %lld outside [1, 2^32]", static_cast<long long>(n_walks));
    if (!std::isfinite(f->scale))
        return fail(MCMF_E_ARG, "scale is not finite");
    if (o) {
        for (uint32_t r : o->reserved)
            if (r != 0)
                return fail(MCMF_E_ARG, "reserved option words must be zero");
        if (o->precision != MCMF_PRECISION_FP64 && o->precision != MCMF_PRECISION_FP32_WEIGHTS)
            return fail(MCMF_E_ARG, "unknown precision %d", o->precision);
        if (!(o->weight_cutoff >= 0.0) || !std::isfinite(o->weight_cutoff))
            return fail(MCMF_E_ARG, "weight_cutoff must be finite and >= 0");
        if (o->allocation != MCMF_ALLOC_PER_ROW && o->allocation != MCMF_ALLOC_NORM &&
            o->allocation != MCMF_ALLOC_NORM_MIN1)
            return fail(MCMF_E_ARG, "unknown allocation %d", o->allocation);
        if (o->allocation != MCMF_ALLOC_PER_ROW && !g->symmetric && g->weighted)
            return fail(MCMF_E_UNSUPPORTED,
                        "MCMF_ALLOC_NORM on a weighted graph needs one created with MCMF_SYMMETRIC");
    }
    return {};
}

namespace {

__global__ void k_col_count(const int32_t *__restrict__ col, int64_t nnz, unsigned int *__restrict__ cnt) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e < nnz)
        atomicAdd(&cnt[col[e]], 1u);
}

// ||C_k||_2 of each start row: along row k (symmetric graphs, in stored
// order, one thread per row) or from the column counts (unweighted).
__global__ void k_start_norms(const int32_t *__restrict__ starts, int64_t n_start,
                              const uint2 *__restrict__ node, const double *__restrict__ val,
                              const unsigned int *__restrict__ colcount, double *__restrict__ out) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n_start)
        return;
    const int32_t k = starts[i];
    double sq = 0.0;
    if (colcount) {
        sq = static_cast<double>(colcount[k]);
    } else {
        const uint2 rk = node[k];
        for (uint32_t j = 0; j < rk.y; ++j) {
            const double a = val ? val[int64_t(rk.x) + j] : 1.0;
            sq = sq + a * a;
        }
    }
    out[i] = sqrt(sq);
}

} // namespace

Status allocate_walks(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t Ns, int K,
                      bool min_one, Allocation &A, hipStream_t s) {
    A.host_starts.clear();
    A.host_walks.clear();
    A.host_rec.assign(1, 0);
    A.n_start = 0;
    A.total = 0;
    A.max_walks = 0;
    if (n_start == 0)
        return {};
    DevBuf<double> norms;
    DevBuf<unsigned int> cnt;
    MCMF_TRY(norms.alloc(n_start, s));
    if (!g->symmetric) {
        MCMF_TRY(cnt.alloc(g->n > 0 ? g->n : 1, s));
        MCMF_TRY(fill_i32(reinterpret_cast<int32_t *>(cnt.ptr), 0, g->n, s));
        if (g->nnz > 0) {
            hipLaunchKernelGGL(k_col_count, dim3(static_cast<uint32_t>((g->nnz + 255) / 256)), dim3(256), 0, s,
                               g->col, g->nnz, cnt.ptr);
            MCMF_HIP(hipGetLastError());
        }
    }
    hipLaunchKernelGGL(k_start_norms, dim3(static_cast<uint32_t>((n_start + 255) / 256)), dim3(256), 0, s,
                       starts, n_start, g->node, g->val, g->symmetric ? nullptr : cnt.ptr, norms.ptr);
    MCMF_HIP(hipGetLastError());
    std::vector<double> hn(static_cast<size_t>(n_start));
    std::vector<int32_t> hs(static_cast<size_t>(n_start));
    MCMF_HIP(hipMemcpyAsync(hn.data(), norms.ptr, sizeof(double) * n_start, hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipMemcpyAsync(hs.data(), starts, sizeof(int32_t) * n_start, hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    double total = 0.0;
    for (double x : hn)
        total = total + x;
    // N_k = N_s p_k rounded half away from zero (Algorithms 2-3); a row
    // rounded to 0 starts no walk and leaves the list.
    int64_t rec = 0;
    for (int64_t i = 0; i < n_start; ++i) {
        int64_t w = total > 0.0 ? std::llround(static_cast<double>(Ns) * (hn[i] / total)) : 0;
        if (min_one)
            w = std::max<int64_t>(w, 1);
        if (w > (int64_t(1) << 31) - 1)
            return fail(MCMF_E_ARG, "MCMF_ALLOC_NORM gives a row %lld walks, above 2^31 - 1",
                        static_cast<long long>(w));
        if (w <= 0)
            continue;
        A.host_starts.push_back(hs[i]);
        A.host_walks.push_back(static_cast<int32_t>(w));
        rec += w * (K - 1);
        A.host_rec.push_back(rec);
        A.total += w;
        A.max_walks = std::max(A.max_walks, w);
    }
    A.n_start = static_cast<int64_t>(A.host_starts.size());
    if (A.n_start == 0)
        return {};
    MCMF_TRY(A.starts.alloc(A.n_start, s));
    MCMF_TRY(A.walks.alloc(A.n_start, s));
    MCMF_TRY(A.rec.alloc(A.n_start + 1, s));
    MCMF_HIP(hipMemcpyAsync(A.starts.ptr, A.host_starts.data(), sizeof(int32_t) * A.n_start,
                            hipMemcpyHostToDevice, s));
    MCMF_HIP(hipMemcpyAsync(A.walks.ptr, A.host_walks.data(), sizeof(int32_t) * A.n_start,
                            hipMemcpyHostToDevice, s));
    MCMF_HIP(hipMemcpyAsync(A.rec.ptr, A.host_rec.data(), sizeof(int64_t) * (A.n_start + 1),
                            hipMemcpyHostToDevice, s));
    // The host vectors must outlive the asynchronous copies.
    MCMF_HIP(hipStreamSynchronize(s));
    return {};
}

// walks_out: the walks per row (0 off the start rows).  Without an
// allocation every row of starts[0..n_start) got N_uniform walks.
Status write_walks_out(const mcmf_graph *g, const int32_t *starts, int64_t n_start, int64_t N_uniform,
                       const Allocation *A, int32_t *walks_out, hipStream_t s) {
    std::vector<int32_t> w(static_cast<size_t>(g->n), 0);
    if (A) {
        for (size_t i = 0; i < A->host_starts.size(); ++i)
            w[static_cast<size_t>(A->host_starts[i])] = A->host_walks[i];
    } else if (n_start > 0) {
        std::vector<int32_t> hs(static_cast<size_t>(n_start));
        MCMF_HIP(hipMemcpyAsync(hs.data(), starts, sizeof(int32_t) * n_start, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipStreamSynchronize(s));
        for (int64_t i = 0; i < n_start; ++i)
            w[static_cast<size_t>(hs[i])] = static_cast<int32_t>(N_uniform);
    }
    if (classify(walks_out) == Mem::Device) {
        if (g->n)
            MCMF_HIP(hipMemcpyAsync(walks_out, w.data(), sizeof(int32_t) * g->n, hipMemcpyHostToDevice, s));
        MCMF_HIP(hipStreamSynchronize(s));
    } else if (g->n) {
        std::copy(w.begin(), w.end(), walks_out);
    }
    return {};
}

namespace {

// Events destroyed on scope exit.
struct EventList : std::vector<hipEvent_t> {
    ~EventList() {
        for (hipEvent_t e : *this)
            if (e)
                (void)hipEventDestroy(e);
    }
};

struct Timer {
    bool on = false;
    hipEvent_t ev[5] = {};
    hipStream_t s = nullptr;
    Status start(bool enable, hipStream_t stream) {
        on = enable;
        s = stream;
        if (!on)
            return {};
        for (auto &e : ev)
            MCMF_HIP(hipEventCreate(&e));
        MCMF_HIP(hipEventRecord(ev[0], s));
        return {};
    }
    Status mark(int i) {
        if (on)
            MCMF_HIP(hipEventRecord(ev[i], s));
        return {};
    }
    float ms(int a, int b) const {
        float t = 0.f;
        if (on && hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) {
            (void)hipGetLastError();
            t = 0.f;
        }
        return t;
    }
    ~Timer() {
        if (on)
            for (auto &e : ev)
                if (e)
                    (void)hipEventDestroy(e);
    }
};


Status run_action(const mcmf_graph *g, const mcmf_fn *f, const double *v, int64_t N, int32_t K,
                  const mcmf_opts *o, double *out, mcmf_stats *stats) {
    MCMF_TRY(check_common(g, f, N, K, o));
    if (!v || !out)
        return fail(MCMF_E_ARG, "v and out must not be NULL");
    if (v == out)
        return fail(MCMF_E_ARG, "out may not alias v");
    std::vector<double> c(K + 1);
    MCMF_TRY(make_coeffs(f, K, c.data()));
    MCMF_HIP(hipSetDevice(g->device));
    hipStream_t s = (o && o->stream) ? static_cast<hipStream_t>(o->stream) : g->stream;
    const int64_t n = g->n;
    uint64_t *digest = o ? o->path_digest : nullptr;
    double *q_out = o ? o->q_out : nullptr;

    Timer tm;
    MCMF_TRY(tm.start(stats != nullptr, s));
    View<double> vin, yout, qv;
    View<uint64_t> dig;
    MCMF_TRY(vin.in(v, n, s));
    MCMF_TRY(yout.out(out, n, s));
    DevBuf<double> rec; // r = s A v
    DevBuf<double> q, coef;
    DevBuf<unsigned long long> steps;
    MCMF_TRY(rec.alloc(n > 0 ? n : 1, s));
    MCMF_TRY(steps.alloc(1, s));
    MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(steps.ptr), 0, 1, s));
    double *qptr = nullptr;
    if (K >= 2) {
        if (q_out && classify(q_out) == Mem::Device) {
            qptr = q_out;
        } else {
            MCMF_TRY(q.alloc(n > 0 ? n : 1, s));
            qptr = q.ptr;
        }
        MCMF_TRY(fill_f64(qptr, 0.0, n, s));
        MCMF_TRY(coef.alloc(K - 1, s));
        MCMF_HIP(hipMemcpyAsync(coef.ptr, c.data() + 2, sizeof(double) * (K - 1),
                                hipMemcpyHostToDevice, s));
    }
    if (digest) {
        MCMF_TRY(dig.out(digest, n, s));
        MCMF_TRY(fill_u64(dig.ptr, 0, n, s));
    }
    MCMF_TRY(tm.mark(1));
    MCMF_TRY(spmv_r(g, vin.ptr, f->scale, rec.ptr, s));
    MCMF_TRY(tm.mark(2));
    const bool by_norm = o && o->allocation != MCMF_ALLOC_PER_ROW && K >= 2;
    Allocation alloc;
    const int32_t *starts = g->active;
    int64_t n_start = K >= 2 ? g->n_active : 0;
    if (by_norm) {
        MCMF_TRY(allocate_walks(g, g->active, g->n_active, N, K, o->allocation == MCMF_ALLOC_NORM_MIN1,
                                alloc, s));
        starts = alloc.starts.ptr;
        n_start = alloc.n_start;
    }
    if (K >= 2) {
        WalkParams p = walk_params(o, coef.ptr, K, f->scale, N);
        if (by_norm)
            p.row_walks = alloc.walks.ptr;
        MCMF_TRY(action_walks(g, rec.ptr, starts, n_start, p, qptr, dig.ptr, steps.ptr, s));
    }
    if (o && o->walks_out)
        MCMF_TRY(write_walks_out(g, starts, n_start, N, by_norm ? &alloc : nullptr, o->walks_out, s));
    MCMF_TRY(tm.mark(3));
    MCMF_TRY(spmv_assemble(g, vin.ptr, rec.ptr, K >= 2 ? qptr : nullptr, c[0], K >= 1 ? c[1] : 0.0,
                           f->scale, yout.ptr, s));
    MCMF_TRY(tm.mark(4));
    MCMF_TRY(yout.copy_back(out, n, s));
    if (digest)
        MCMF_TRY(dig.copy_back(digest, n, s));
    if (q_out) {
        if (K < 2) {
            if (classify(q_out) == Mem::Device)
                MCMF_TRY(fill_f64(q_out, 0.0, n, s));
            else
                std::fill(q_out, q_out + n, 0.0); // nothing was estimated
        } else if (qptr != q_out && n) {
            MCMF_HIP(hipMemcpyAsync(q_out, qptr, sizeof(double) * n, hipMemcpyDeviceToHost, s));
        }
    }
    const bool sync = !(o && o->stream) || stats || vin.host || yout.host ||
                      (digest && dig.host) || (q_out && classify(q_out) == Mem::Host);
    unsigned long long nsteps = 0;
    if (stats)
        MCMF_HIP(hipMemcpyAsync(&nsteps, steps.ptr, sizeof nsteps, hipMemcpyDeviceToHost, s));
    if (sync)
        MCMF_HIP(hipStreamSynchronize(s));
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->start_rows = static_cast<uint64_t>(n_start);
        stats->walks = by_norm ? static_cast<uint64_t>(alloc.total)
                               : stats->start_rows * static_cast<uint64_t>(K >= 2 ? N : 0);
        stats->walk_steps = nsteps;
        stats->ms_setup = tm.ms(0, 1);
        stats->ms_spmv = tm.ms(1, 2) + tm.ms(3, 4);
        stats->ms_walk = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 4);
    }
    return {};
}

Status run_diag(const mcmf_graph *g, const mcmf_fn *f, const int32_t *rows, int64_t n_rows,
                int64_t N, int32_t K, const mcmf_opts *o, double *out, mcmf_stats *stats) {
    MCMF_TRY(check_common(g, f, N, K, o));
    if (!out)
        return fail(MCMF_E_ARG, "out must not be NULL");
    if (rows && n_rows < 0)
        return fail(MCMF_E_ARG, "n_rows = %lld is negative", static_cast<long long>(n_rows));
    if (!g->symmetric)
        return fail(MCMF_E_NOT_SYMMETRIC, "mcmf_diag needs a graph created with MCMF_SYMMETRIC");
    const bool all = rows == nullptr;
    const int64_t count = all ? g->n : n_rows;
    if (!all && classify(rows) == Mem::Host)
        for (int64_t p = 0; p < n_rows; ++p)
            if (rows[p] < 0 || rows[p] >= g->n)
                return fail(MCMF_E_ARG, "rows[%lld] = %d outside [0, %lld)", static_cast<long long>(p),
                            rows[p], static_cast<long long>(g->n));
    std::vector<double> c(K + 1);
    MCMF_TRY(make_coeffs(f, K, c.data()));
    MCMF_HIP(hipSetDevice(g->device));
    hipStream_t s = (o && o->stream) ? static_cast<hipStream_t>(o->stream) : g->stream;
    const int64_t n = g->n;
    uint64_t *digest = o ? o->path_digest : nullptr;

    Timer tm;
    MCMF_TRY(tm.start(stats != nullptr, s));
    View<int32_t> rv;
    View<double> dout;
    View<uint64_t> dig;
    if (!all)
        MCMF_TRY(rv.in(rows, count, s));
    MCMF_TRY(dout.out(out, count, s));
    DevBuf<double> dacc, coef;
    DevBuf<uint8_t> in_set, start_flags;
    DevBuf<int32_t> start_list;
    DevBuf<int> bad;
    DevBuf<unsigned long long> counters; // steps, probes, table overflows
    MCMF_TRY(counters.alloc(3, s));
    MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(counters.ptr), 0, 3, s));
    if (digest) {
        MCMF_TRY(dig.out(digest, n, s));
        MCMF_TRY(fill_u64(dig.ptr, 0, n, s));
    }
    const int32_t *starts = g->active;
    int64_t n_start = g->n_active;
    if (!all) {
        // Rows given in device memory are range-checked here, before any write to out.
        MCMF_TRY(in_set.alloc(n > 0 ? n : 1, s));
        MCMF_TRY(bad.alloc(1, s));
        MCMF_TRY(fill_u8(in_set.ptr, 0, n, s));
        MCMF_TRY(fill_i32(bad.ptr, 0, 1, s));
        if (count > 0) {
            hipLaunchKernelGGL(k_mark_rows, dim3(grid_for(count, 256)), dim3(256), 0, s, rv.ptr, count,
                               n, in_set.ptr, bad.ptr);
            MCMF_HIP(hipGetLastError());
        }
        int hbad = 0;
        MCMF_HIP(hipMemcpyAsync(&hbad, bad.ptr, sizeof hbad, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipStreamSynchronize(s));
        if (hbad)
            return fail(MCMF_E_ARG, "a requested row lies outside [0, %lld)", static_cast<long long>(n));
        n_start = 0;
        if (K >= 2 && count > 0) {
            MCMF_TRY(start_flags.alloc(n > 0 ? n : 1, s));
            MCMF_TRY(start_list.alloc(n > 0 ? n : 1, s));
            MCMF_TRY(fill_u8(start_flags.ptr, 0, n, s));
            hipLaunchKernelGGL(k_mark_starts, dim3(grid_for(count, 4)), dim3(256), 0, s, rv.ptr, count,
                               g->node, g->col, start_flags.ptr);
            MCMF_HIP(hipGetLastError());
            MCMF_TRY(compact(start_flags.ptr, n, 1, start_list.ptr, &n_start, s));
        }
        starts = start_list.ptr;
    }
    // Walks per start row by column norm: rows allocated none leave the list.
    const bool by_norm = o && o->allocation != MCMF_ALLOC_PER_ROW && K >= 2;
    Allocation alloc;
    if (by_norm) {
        MCMF_TRY(allocate_walks(g, starts, n_start, N, K, o->allocation == MCMF_ALLOC_NORM_MIN1, alloc, s));
        starts = alloc.starts.ptr;
        n_start = alloc.n_start;
    }
    // Work items of the gather over the start list.
    DevBuf<int64_t> item_buf;
    const int64_t *item_off = g->active_items;
    if ((!all || by_norm) && K >= 2 && n_start > 0) {
        MCMF_TRY(item_buf.alloc(n_start + 1, s));
        MCMF_TRY(gather_items(g, starts, n_start, item_buf.ptr, s));
        item_off = item_buf.ptr;
    }
    if (K >= 2) {
        MCMF_TRY(dacc.alloc(n > 0 ? n : 1, s));
        MCMF_TRY(fill_f64(dacc.ptr, 0.0, n, s));
        MCMF_TRY(coef.alloc(K - 1, s));
        MCMF_HIP(hipMemcpyAsync(coef.ptr, c.data() + 2, sizeof(double) * (K - 1),
                                hipMemcpyHostToDevice, s));
    }
    MCMF_TRY(tm.mark(1));
    float ms_walk = 0.f, ms_gather = 0.f;
    EventList chunk_events;
    // A call that returns before its work is done records a Q_k table
    // overflow (a planning error) on the graph, for the next synchronising
    // call to report; a synchronising call checks its own counter.
    const bool sync = !(o && o->stream) || stats || dout.host || (digest && dig.host) || rv.host;
    if (o && o->walks_out)
        MCMF_TRY(write_walks_out(g, starts, K >= 2 ? n_start : 0, N, by_norm ? &alloc : nullptr,
                                 o->walks_out, s));
    if (K >= 2 && n_start > 0) {
        WalkParams p = walk_params(o, coef.ptr, K, f->scale, N);
        if (by_norm) {
            // The gather indexes the whole start list; its table is planned
            // for the row with the most walks.
            p.row_walks = alloc.walks.ptr;
            p.row_rec = alloc.rec.ptr;
            p.n_walks = alloc.max_walks;
        }
        // Hub rows: the walks sum them, the gather leaves them out.
        if (wide_diag(g, p))
            p.whub_act = active_wide_hubs(g, p.n_walks, K);
        else
            p.hub_act = g->weighted ? 0u : active_hubs(g, p.n_walks, K);
        p.in_set = all ? nullptr : in_set.ptr;
        p.dacc = dacc.ptr;
        // Visit records of a chunk of start rows: 12 bytes per visit (8 with
        // FP32 walk weights).  Chunk boundaries: rows [bounds[i], bounds[i+1]).
        const int64_t per_row = N * (K - 1);
        const int64_t xbytes = p.precision == MCMF_PRECISION_FP32_WEIGHTS ? 4 : 8;
        std::vector<int64_t> bounds;
        int64_t most_recs = 0;
        auto plan_chunks = [&](int64_t chunk_recs) {
            bounds.assign(1, 0);
            most_recs = 0;
            if (by_norm) {
                int64_t c0 = 0;
                while (c0 < n_start) {
                    int64_t c1 = c0 + 1; // at least one row per chunk
                    while (c1 < n_start && alloc.host_rec[c1 + 1] - alloc.host_rec[c0] <= chunk_recs)
                        ++c1;
                    most_recs = std::max(most_recs, alloc.host_rec[c1] - alloc.host_rec[c0]);
                    bounds.push_back(c1);
                    c0 = c1;
                }
            } else {
                int64_t rows_per_chunk = std::max<int64_t>(1, std::min<int64_t>(chunk_recs / per_row, n_start));
                for (int64_t c0 = rows_per_chunk; c0 < n_start; c0 += rows_per_chunk)
                    bounds.push_back(c0);
                bounds.push_back(n_start);
                most_recs = rows_per_chunk * per_row;
            }
        };
        DevBuf<int32_t> vstate;
        DevBuf<unsigned char> vx;
        // The default buffer is halved while device memory (or the byte
        // budget) refuses it; an explicit MCMF_DIAG_CHUNK_BYTES is kept.
        for (int64_t chunk_bytes = default_visit_chunk_bytes();; chunk_bytes /= 2) {
            plan_chunks(std::max<int64_t>(1, chunk_bytes / (4 + xbytes)));
            Status st = vstate.alloc(most_recs, s);
            if (!st)
                st = vx.alloc(most_recs * xbytes, s);
            if (!st)
                break;
            vstate.reset();
            vx.reset();
            if (st.code != MCMF_E_NOMEM || visit_chunk_bytes_fixed() || chunk_bytes / 2 < kMinVisitChunkBytes)
                return st;
            clear_error();
        }
        // Per-chunk events are read only after the call's final synchronisation,
        // so timing does not stall the stream between chunks.
        const int64_t n_chunks = static_cast<int64_t>(bounds.size()) - 1;
        DevBuf<unsigned long long> queues; // one work counter per gather launch
        MCMF_TRY(queues.alloc(n_chunks, s));
        MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(queues.ptr), 0, n_chunks, s));
        if (stats) {
            chunk_events.assign(static_cast<size_t>(2 * n_chunks + 1), nullptr);
            for (auto &e : chunk_events)
                MCMF_HIP(hipEventCreate(&e));
        }
        for (int64_t ci = 0; ci < n_chunks; ++ci) {
            const int64_t c0 = bounds[ci];
            const int64_t rows_here = bounds[ci + 1] - c0;
            if (stats)
                MCMF_HIP(hipEventRecord(chunk_events[2 * ci], s));
            WalkParams pw = p; // the walk launch indexes this chunk's rows
            if (by_norm) {
                pw.row_walks = alloc.walks.ptr + c0;
                pw.row_rec = alloc.rec.ptr + c0;
            }
            MCMF_TRY(diag_walks(g, starts + c0, rows_here, pw, vstate.ptr, vx.ptr, dig.ptr,
                                counters.ptr, s));
            if (stats)
                MCMF_HIP(hipEventRecord(chunk_events[2 * ci + 1], s));
            MCMF_TRY(diag_gather(g, starts, item_off, c0, c0 + rows_here, p, vstate.ptr, vx.ptr,
                                 all ? nullptr : in_set.ptr, dacc.ptr, counters.ptr + 1,
                                 sync ? counters.ptr + 2 : g->async_overflow, queues.ptr + ci, s));
        }
        if (stats)
            MCMF_HIP(hipEventRecord(chunk_events.back(), s));
    }
    MCMF_TRY(tm.mark(2));
    if (count > 0) {
        hipLaunchKernelGGL(k_diag_finish, dim3(grid_for(count, 4)), dim3(256), 0, s,
                           all ? nullptr : rv.ptr, count, g->node, g->col, g->val, K, c[0],
                           K >= 1 ? c[1] : 0.0, f->scale, dacc.ptr, dout.ptr);
        MCMF_HIP(hipGetLastError());
    }
    MCMF_TRY(tm.mark(3));
    MCMF_TRY(dout.copy_back(out, count, s));
    if (digest)
        MCMF_TRY(dig.copy_back(digest, n, s));
    unsigned long long hc[3] = {0, 0, 0}, earlier = 0;
    if (sync) {
        MCMF_HIP(hipMemcpyAsync(hc, counters.ptr, sizeof hc, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipMemcpyAsync(&earlier, g->async_overflow, sizeof earlier, hipMemcpyDeviceToHost, s));
        MCMF_HIP(hipStreamSynchronize(s));
    }
    if (hc[2] != 0)
        return fail(MCMF_E_DEVICE, "internal error: a Q_k table overflowed (%llu inserts lost)", hc[2]);
    if (earlier != 0) {
        MCMF_TRY(fill_u64(reinterpret_cast<uint64_t *>(g->async_overflow), 0, 1, s));
        MCMF_HIP(hipStreamSynchronize(s));
        return fail(MCMF_E_DEVICE,
                    "internal error: a Q_k table of an earlier asynchronous mcmf_diag on this graph "
                    "overflowed (%llu inserts lost)", earlier);
    }
    if (stats) {
        for (size_t e = 0; e + 1 < chunk_events.size(); ++e) {
            float t = 0.f;
            MCMF_HIP(hipEventElapsedTime(&t, chunk_events[e], chunk_events[e + 1]));
            // even -> odd: walk kernel; odd -> next even: gather kernel
            if (e % 2 == 0)
                ms_walk += t;
            else
                ms_gather += t;
        }
        memset(stats, 0, sizeof *stats);
        stats->start_rows = K >= 2 ? static_cast<uint64_t>(n_start) : 0;
        stats->walks = by_norm ? static_cast<uint64_t>(alloc.total)
                               : stats->start_rows * static_cast<uint64_t>(K >= 2 ? N : 0);
        stats->walk_steps = hc[0];
        stats->gather_probes = hc[1];
        stats->ms_setup = tm.ms(0, 1);
        stats->ms_walk = ms_walk;
        stats->ms_gather = ms_gather;
        stats->ms_spmv = tm.ms(2, 3);
        stats->ms_total = tm.ms(0, 3);
    }
    return {};
}

} // namespace

} // namespace mcmf

using namespace mcmf;

extern "C" mcmf_status mcmf_action(const mcmf_graph *g, const mcmf_fn *f, const double *v,
                                   int64_t n_walks, int32_t K, const mcmf_opts *opts, double *out,
                                   mcmf_stats *stats) {
    clear_error();
    return run_action(g, f, v, n_walks, K, opts, out, stats).code;
}

extern "C" mcmf_status mcmf_diag(const mcmf_graph *g, const mcmf_fn *f, const int32_t *rows,
                                 int64_t n_rows, int64_t n_walks, int32_t K, const mcmf_opts *opts,
                                 double *out, mcmf_stats *stats) {
    clear_error();
    return run_diag(g, f, rows, n_rows, n_walks, K, opts, out, stats).code;
}
