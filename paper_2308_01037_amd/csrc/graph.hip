// CSR graph store in device memory and its per-row metadata (row records,
// rows with entries, length bins, |a| sums and running sums for weighted
// rows), plus the small utility kernels (fills, ordered compaction).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "device.hpp"
#include "ops.hpp"

namespace mcmf {

namespace {

constexpr int kThreads = 256;
// Column array plus row records up to which the diagonal walk defaults to
// the ROW layout.
constexpr int64_t kRowLayoutBytes = int64_t(16) << 20;

int64_t grid_for(int64_t n, int threads = kThreads, int64_t cap = 1 << 20) {
    int64_t b = (n + threads - 1) / threads;
    if (b < 1)
        b = 1;
    return b < cap ? b : cap;
}

template <class T>
__global__ void k_fill(T *out, T value, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        out[i] = value;
}

template <class T>
Status fill_impl(T *out, T value, int64_t n, hipStream_t s) {
    if (n <= 0)
        return {};
    hipLaunchKernelGGL(k_fill<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, out, value, n);
    MCMF_HIP(hipGetLastError());
    return {};
}

// ---- ordered compaction: 256 threads x 16 consecutive flags per block ----

constexpr int kCompactPer = 16;
constexpr int kCompactSpan = kThreads * kCompactPer;

__device__ __forceinline__ uint32_t count_run(const uint8_t *flags, int64_t n, uint8_t match,
                                              int64_t first) {
    uint32_t c = 0;
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
        const int64_t i = first + j;
        c += (i < n && flags[i] == match) ? 1u : 0u;
    }
    return c;
}

__global__ __launch_bounds__(kThreads) void k_compact_count(const uint8_t *flags, int64_t n,
                                                            uint8_t match, uint32_t *counts) {
    __shared__ uint32_t scratch[kThreads / 64];
    const int64_t first = int64_t(blockIdx.x) * kCompactSpan + int64_t(threadIdx.x) * kCompactPer;
    const uint32_t c = count_run(flags, n, match, first);
    uint32_t total = 0;
    dev::block_exclusive_scan(c, scratch, &total);
    if (threadIdx.x == 0)
        counts[blockIdx.x] = total;
}

// One workgroup turns the per-block counts into exclusive offsets.
__global__ __launch_bounds__(1024) void k_compact_scan(uint32_t *counts, int64_t nb,
                                                       unsigned long long *total) {
    __shared__ uint32_t scratch[1024 / 64];
    uint64_t running = 0;
    for (int64_t base = 0; base < nb; base += blockDim.x) {
        const int64_t i = base + threadIdx.x;
        const uint32_t c = i < nb ? counts[i] : 0u;
        uint32_t chunk = 0;
        const uint32_t ex = dev::block_exclusive_scan(c, scratch, &chunk);
        if (i < nb)
            counts[i] = static_cast<uint32_t>(running + ex);
        running += chunk;
    }
    if (threadIdx.x == 0)
        *total = running;
}

__global__ __launch_bounds__(kThreads) void k_compact_write(const uint8_t *flags, int64_t n,
                                                            uint8_t match, const uint32_t *offsets,
                                                            int32_t *out) {
    __shared__ uint32_t scratch[kThreads / 64];
    const int64_t first = int64_t(blockIdx.x) * kCompactSpan + int64_t(threadIdx.x) * kCompactPer;
    const uint32_t c = count_run(flags, n, match, first);
    uint32_t total = 0;
    uint32_t pos = offsets[blockIdx.x] + dev::block_exclusive_scan(c, scratch, &total);
    for (int j = 0; j < kCompactPer; ++j) {
        const int64_t i = first + j;
        if (i < n && flags[i] == match)
            out[pos++] = static_cast<int32_t>(i);
    }
}

// ---- graph construction ----

enum : int {
    kErrRowPtr = 1,    // decreasing row_ptr
    kErrColumn = 2,    // column outside [0, n)
    kErrValue = 4,     // non-finite value
    kErrUnsorted = 8,  // row not strictly increasing (symmetry check, hub rows)
    kErrAsymmetric = 16,
};

__global__ void k_check_row_ptr(const int64_t *row_ptr, int64_t n, int *err) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        if (row_ptr[i + 1] < row_ptr[i])
            atomicOr(err, kErrRowPtr);
}

// One wavefront per row: column range, finite values, and strict order.
__global__ __launch_bounds__(kThreads) void k_check_entries(const int64_t *row_ptr, int64_t n,
                                                            const int32_t *col, const double *val,
                                                            int *err) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / 64);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6); i < n; i += waves) {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        int bad = 0;
        for (int64_t k = b + lane; k < e; k += 64) {
            const int32_t c = col[k];
            if (c < 0 || c >= n)
                bad |= kErrColumn;
            if (val && !isfinite(val[k]))
                bad |= kErrValue;
            if (k + 1 < e && col[k + 1] <= c)
                bad |= kErrUnsorted;
        }
        if (bad)
            atomicOr(err, bad);
    }
}

// Per-row metadata.  Weighted rows get sum |a| and the running sums of |a|
// in storage order, each a plain left-to-right FP64 sum.
__global__ void k_graph_meta(const int64_t *row_ptr, int64_t n, const double *val, uint2 *node,
                             uint8_t *active, uint8_t *bin, double *rowabs, double *cum,
                             unsigned long long *dmax) {
    unsigned long long local_max = 0;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int64_t b = row_ptr[i], e = row_ptr[i + 1];
        const int64_t d = e - b;
        node[i] = make_uint2(static_cast<uint32_t>(b), static_cast<uint32_t>(d));
        active[i] = d > 0 ? 1 : 0;
        bin[i] = d <= 64 ? 0 : (d <= 4096 ? 1 : 2);
        local_max = d > static_cast<int64_t>(local_max) ? static_cast<unsigned long long>(d) : local_max;
        if (val) {
            double sum = 0.0;
            for (int64_t k = b; k < e; ++k) {
                sum = sum + fabs(val[k]);
                cum[k] = sum;
            }
            rowabs[i] = sum;
        }
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long other = __shfl_xor(local_max, off, 64);
        local_max = other > local_max ? other : local_max;
    }
    if ((threadIdx.x & 63) == 0)
        atomicMax(dmax, local_max);
}

// edge[e] = {col[e], record of row col[e], hubs adjacent to col[e]} for
// every stored entry (hubmask null: no hubs).
__global__ void k_build_edges(const int32_t *col, int64_t nnz, const uint2 *node,
                              const uint32_t *hubmask, uint4 *edge) {
    for (int64_t e = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; e < nnz;
         e += int64_t(gridDim.x) * blockDim.x) {
        const int32_t j = col[e];
        const uint2 rj = node[j];
        edge[e] = make_uint4(static_cast<uint32_t>(j), rj.x, rj.y, hubmask ? hubmask[j] : 0u);
    }
}

// Hub h (one workgroup each): bit h in the mask of every column of its row.
__global__ void k_hub_marks(const int32_t *hub_rows, const uint2 *node, const int32_t *col,
                            uint32_t *hubmask, uint8_t *hub_of) {
    const int h = blockIdx.x;
    const int32_t row = hub_rows[h];
    const uint2 r = node[row];
    for (uint32_t e = threadIdx.x; e < r.y; e += blockDim.x)
        atomicOr(&hubmask[col[int64_t(r.x) + e]], 1u << h);
    if (threadIdx.x == 0)
        hub_of[row] = static_cast<uint8_t>(h);
}

// Wide hub h (one workgroup each): its bit in the wide mask of every column
// of its row.
__global__ void k_whub_marks(const int32_t *whub_rows, const uint2 *node, const int32_t *col,
                             uint32_t *wmask, uint16_t *whub_of) {
    const int h = blockIdx.x;
    const int32_t row = whub_rows[h];
    const uint2 r = node[row];
    for (uint32_t e = threadIdx.x; e < r.y; e += blockDim.x)
        atomicOr(&wmask[int64_t(col[int64_t(r.x) + e]) * kWideWords + h / 32], 1u << (h % 32));
    if (threadIdx.x == 0)
        whub_of[row] = static_cast<uint16_t>(h);
}

// a_ji == a_ij for every stored a_ij (rows sorted): one wavefront per row,
// each lane binary-searches row j for i.
__global__ __launch_bounds__(kThreads) void k_check_symmetric(const uint2 *node, int64_t n,
                                                              const int32_t *col, const double *val,
                                                              int *err) {
    const int lane = threadIdx.x & 63;
    const int64_t waves = int64_t(gridDim.x) * (blockDim.x / 64);
    for (int64_t i = blockIdx.x * int64_t(blockDim.x / 64) + (threadIdx.x >> 6); i < n; i += waves) {
        const uint2 ri = node[i];
        int bad = 0;
        for (uint32_t k = lane; k < ri.y; k += 64) {
            const int64_t e = int64_t(ri.x) + k;
            const int32_t j = col[e];
            const uint2 rj = node[j];
            uint32_t lo = 0, hi = rj.y;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (col[int64_t(rj.x) + mid] < i)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            if (lo >= rj.y || col[int64_t(rj.x) + lo] != i)
                bad = kErrAsymmetric;
            else if (val && val[int64_t(rj.x) + lo] != val[e])
                bad = kErrAsymmetric;
        }
        if (bad)
            atomicOr(err, bad);
    }
}

Status read_scalar(const int64_t *p, int64_t *out, Mem m) {
    if (m == Mem::Host) {
        *out = *p;
        return {};
    }
    MCMF_HIP(hipMemcpy(out, p, sizeof(int64_t), hipMemcpyDeviceToHost));
    return {};
}

Status copy_in(void *dst, const void *src, size_t bytes, Mem m, hipStream_t s) {
    if (bytes == 0)
        return {};
    MCMF_HIP(hipMemcpyAsync(dst, src, bytes,
                            m == Mem::Host ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice, s));
    return {};
}

Status read_flag(int *dflag, int *out, hipStream_t s) {
    MCMF_HIP(hipMemcpyAsync(out, dflag, sizeof(int), hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    return {};
}

void free_graph(mcmf_graph *g) {
    if (!g)
        return;
    if (g->stream)
        (void)hipStreamSynchronize(g->stream);
    dev_free_sync(g->col, sizeof(int32_t) * g->nnz);
    dev_free_sync(g->val, sizeof(double) * g->nnz);
    dev_free_sync(g->rowabs, sizeof(double) * g->n);
    dev_free_sync(g->cum, sizeof(double) * g->nnz);
    dev_free_sync(g->alias_rec, sizeof(uint4) * g->nnz);
    dev_free_sync(g->node, sizeof(uint2) * g->n);
    dev_free_sync(g->edge, sizeof(uint4) * g->nnz);
    dev_free_sync(g->active, sizeof(int32_t) * g->n_active);
    dev_free_sync(g->active_items, sizeof(int64_t) * (g->n_active + 1));
    dev_free_sync(g->bin_rows, sizeof(int32_t) * g->n);
    dev_free_sync(g->hubmask, sizeof(uint32_t) * g->n);
    dev_free_sync(g->hub_of, sizeof(uint8_t) * g->n);
    dev_free_sync(g->hub_rows, sizeof(int32_t) * kMaxHubs);
    dev_free_sync(g->whub_rows, sizeof(int32_t) * g->n_whubs);
    dev_free_sync(g->whub_of, sizeof(uint16_t) * g->n);
    dev_free_sync(g->wmask, sizeof(uint32_t) * kWideWords * g->n);
    dev_free_sync(g->async_overflow, sizeof(unsigned long long));
    if (g->stream)
        (void)hipStreamDestroy(g->stream);
    delete g;
}

// The graph's hub rows: the kMaxWideHubs rows of largest degree (ties:
// lower row first), chosen on the host from the row records.  The first
// kMaxHubs are the hubs of the 32-bit masks (every edge record's spare word);
// when there are more, all of them get wide masks if those fit 1/32 of
// device memory.
Status build_hubs(mcmf_graph *g, hipStream_t s) {
    const int64_t n = g->n;
    std::vector<uint2> node(static_cast<size_t>(n));
    MCMF_HIP(hipMemcpyAsync(node.data(), g->node, sizeof(uint2) * n, hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    std::vector<std::pair<uint32_t, int32_t>> top; // (degree, row), degree descending
    auto before = [](const std::pair<uint32_t, int32_t> &a, const std::pair<uint32_t, int32_t> &b) {
        return a.first > b.first;
    };
    for (int64_t i = 0; i < n; ++i) {
        const uint32_t d = node[static_cast<size_t>(i)].y;
        if (d == 0 || (static_cast<int>(top.size()) == kMaxWideHubs && d <= top.back().first))
            continue;
        const std::pair<uint32_t, int32_t> x(d, static_cast<int32_t>(i));
        top.insert(std::upper_bound(top.begin(), top.end(), x, before), x);
        if (static_cast<int>(top.size()) > kMaxWideHubs)
            top.pop_back();
    }
    g->n_hubs = static_cast<int32_t>(std::min<size_t>(top.size(), kMaxHubs));
    if (g->n_hubs == 0)
        return {};
    for (int h = 0; h < g->n_hubs; ++h) {
        g->hub_rows_host[h] = top[h].second;
        g->hub_deg_host[h] = top[h].first;
    }
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->hubmask), sizeof(uint32_t) * n));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->hub_of), sizeof(uint8_t) * n));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->hub_rows), sizeof(int32_t) * kMaxHubs));
    MCMF_TRY(fill_impl<uint32_t>(g->hubmask, 0u, n, s));
    MCMF_TRY(fill_impl<uint8_t>(g->hub_of, kNoHub, n, s));
    MCMF_HIP(hipMemcpyAsync(g->hub_rows, g->hub_rows_host, sizeof(int32_t) * kMaxHubs,
                            hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_hub_marks, dim3(g->n_hubs), dim3(kThreads), 0, s, g->hub_rows, g->node, g->col,
                       g->hubmask, g->hub_of);
    MCMF_HIP(hipGetLastError());
    const uint64_t wide_bytes = (sizeof(uint32_t) * kWideWords + sizeof(uint16_t)) * static_cast<uint64_t>(n);
    if (top.size() > static_cast<size_t>(kMaxHubs) && wide_bytes <= device_memory_bytes() / 32) {
        g->n_whubs = static_cast<int32_t>(top.size());
        g->whub_deg_host.resize(top.size());
        g->whub_sq_prefix.assign(top.size() + 1, 0.0);
        std::vector<int32_t> rows(top.size());
        for (size_t h = 0; h < top.size(); ++h) {
            rows[h] = top[h].second;
            g->whub_deg_host[h] = top[h].first;
            const double d = static_cast<double>(top[h].first);
            g->whub_sq_prefix[h + 1] = g->whub_sq_prefix[h] + d * d;
        }
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->whub_rows), sizeof(int32_t) * g->n_whubs));
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->whub_of), sizeof(uint16_t) * n));
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->wmask), sizeof(uint32_t) * kWideWords * n));
        MCMF_TRY(fill_impl<uint32_t>(g->wmask, 0u, kWideWords * n, s));
        MCMF_TRY(fill_impl<uint16_t>(g->whub_of, kNoWideHub, n, s));
        MCMF_HIP(hipMemcpyAsync(g->whub_rows, rows.data(), sizeof(int32_t) * g->n_whubs, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_whub_marks, dim3(g->n_whubs), dim3(kThreads), 0, s, g->whub_rows, g->node, g->col,
                           g->wmask, g->whub_of);
        MCMF_HIP(hipGetLastError());
    }
    MCMF_HIP(hipStreamSynchronize(s));
    return {};
}

Status build_graph(mcmf_graph *g, int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const double *values, uint32_t flags) {
    const Mem m_rp = classify(row_ptr);
    const Mem m_col = classify(col);
    const Mem m_val = classify(values);
    int64_t first = 0, nnz = 0;
    MCMF_TRY(read_scalar(row_ptr, &first, m_rp));
    MCMF_TRY(read_scalar(row_ptr + n, &nnz, m_rp));
    if (first != 0)
        return fail(MCMF_E_CSR, "row_ptr[0] = %lld, expected 0", static_cast<long long>(first));
    if (nnz < 0)
        return fail(MCMF_E_CSR, "row_ptr[n] = %lld is negative", static_cast<long long>(nnz));
    if (nnz >= (int64_t(1) << 32))
        return fail(MCMF_E_UNSUPPORTED, "nnz = %lld: at most 2^32-1 entries are supported",
                    static_cast<long long>(nnz));
    if (nnz > 0 && !col)
        return fail(MCMF_E_ARG, "col_idx is NULL with nnz > 0");

    MCMF_HIP(hipGetDevice(&g->device));
    MCMF_HIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
    hipStream_t s = g->stream;
    g->n = n;
    g->nnz = nnz;
    g->weighted = values != nullptr;
    g->symmetric = (flags & MCMF_SYMMETRIC) != 0;

    DevBuf<int64_t> d_rp;
    DevBuf<int> d_err;
    DevBuf<unsigned long long> d_dmax;
    DevBuf<uint8_t> d_active, d_bin;
    MCMF_TRY(d_rp.alloc(n + 1, s));
    MCMF_TRY(d_err.alloc(1, s));
    MCMF_TRY(d_dmax.alloc(1, s));
    MCMF_TRY(d_active.alloc(n > 0 ? n : 1, s));
    MCMF_TRY(d_bin.alloc(n > 0 ? n : 1, s));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->col), sizeof(int32_t) * nnz));
    if (g->weighted) {
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->val), sizeof(double) * nnz));
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->cum), sizeof(double) * nnz));
        MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->rowabs), sizeof(double) * n));
    }
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->node), sizeof(uint2) * n));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->edge), sizeof(uint4) * nnz));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->bin_rows), sizeof(int32_t) * n));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->async_overflow), sizeof(unsigned long long)));
    MCMF_TRY(fill_impl<unsigned long long>(g->async_overflow, 0ull, 1, s));

    MCMF_TRY(copy_in(d_rp.ptr, row_ptr, sizeof(int64_t) * (n + 1), m_rp, s));
    MCMF_TRY(copy_in(g->col, col, sizeof(int32_t) * nnz, m_col, s));
    if (g->weighted)
        MCMF_TRY(copy_in(g->val, values, sizeof(double) * nnz, m_val, s));

    // Structure first: a decreasing row_ptr would send the entry checks out of range.
    int err = 0;
    MCMF_TRY(fill_impl<int>(d_err.ptr, 0, 1, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_check_row_ptr, dim3(grid_for(n)), dim3(kThreads), 0, s, d_rp.ptr, n,
                           d_err.ptr);
        MCMF_HIP(hipGetLastError());
    }
    MCMF_TRY(read_flag(d_err.ptr, &err, s));
    if (err & kErrRowPtr)
        return fail(MCMF_E_CSR, "row_ptr is not non-decreasing");
    const bool validate = (flags & MCMF_VALIDATE) != 0;
    const bool check_sym = validate && g->symmetric;
    if (n > 0) {
        hipLaunchKernelGGL(k_check_entries, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, d_rp.ptr,
                           n, g->col, validate ? g->val : nullptr, d_err.ptr);
        MCMF_HIP(hipGetLastError());
    }
    MCMF_TRY(read_flag(d_err.ptr, &err, s));
    if (err & kErrColumn)
        return fail(MCMF_E_CSR, "a column index lies outside [0, n)");
    if (err & kErrValue)
        return fail(MCMF_E_CSR, "a stored value is not finite");
    g->strict_rows = (err & kErrUnsorted) == 0;
    if (check_sym && (err & kErrUnsorted))
        return fail(MCMF_E_NOT_SYMMETRIC,
                    "the symmetry check needs strictly increasing columns within each row");

    MCMF_TRY(fill_impl<unsigned long long>(d_dmax.ptr, 0ull, 1, s));
    if (n > 0) {
        hipLaunchKernelGGL(k_graph_meta, dim3(grid_for(n)), dim3(kThreads), 0, s, d_rp.ptr, n,
                           g->val, g->node, d_active.ptr, d_bin.ptr, g->rowabs, g->cum, d_dmax.ptr);
        MCMF_HIP(hipGetLastError());
    }
    if (!g->weighted && g->symmetric && g->strict_rows && nnz > 0)
        MCMF_TRY(build_hubs(g, s));
    if (nnz > 0) {
        hipLaunchKernelGGL(k_build_edges, dim3(grid_for(nnz)), dim3(kThreads), 0, s, g->col, nnz,
                           g->node, g->hubmask, g->edge);
        MCMF_HIP(hipGetLastError());
    }
    if (check_sym && n > 0) {
        hipLaunchKernelGGL(k_check_symmetric, dim3(grid_for(n, 4)), dim3(kThreads), 0, s, g->node,
                           n, g->col, g->val, d_err.ptr);
        MCMF_HIP(hipGetLastError());
        MCMF_TRY(read_flag(d_err.ptr, &err, s));
        if (err & kErrAsymmetric)
            return fail(MCMF_E_NOT_SYMMETRIC, "A is not equal to its transpose");
    }
    unsigned long long dmax = 0;
    MCMF_HIP(hipMemcpyAsync(&dmax, d_dmax.ptr, sizeof dmax, hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    g->d_max = static_cast<int64_t>(dmax);
    // Default layout of the diagonal walk: while the column array and the
    // row records are small enough to stay in cache, the ROW step (4-byte
    // column, then the 8-byte row record) beats the 16-byte EDGE record.  On
    // R-MAT graphs the walk was 23% faster with ROW at 8 MB of column array
    // and row records, 6% at 16 MB, and 16% slower at 32 MB.
    if (!g->weighted && 4 * nnz + 8 * n <= kRowLayoutBytes)
        g->tuning.diag_sampler = MCMF_SAMPLER_ROW;

    // Rows with entries (walk start rows), then rows by length bin.
    DevBuf<int32_t> tmp_active;
    MCMF_TRY(tmp_active.alloc(n > 0 ? n : 1, s));
    MCMF_TRY(compact(d_active.ptr, n, 1, tmp_active.ptr, &g->n_active, s));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->active), sizeof(int32_t) * g->n_active));
    if (g->n_active > 0)
        MCMF_HIP(hipMemcpyAsync(g->active, tmp_active.ptr, sizeof(int32_t) * g->n_active,
                                hipMemcpyDeviceToDevice, s));
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&g->active_items),
                            sizeof(int64_t) * (g->n_active + 1)));
    MCMF_TRY(gather_items(g, g->active, g->n_active, g->active_items, s));
    int64_t off = 0;
    for (int b = 0; b < 3; ++b) {
        g->bin_offset[b] = off;
        MCMF_TRY(compact(d_bin.ptr, n, static_cast<uint8_t>(b), g->bin_rows + off, &g->bin_count[b], s));
        off += g->bin_count[b];
    }
    MCMF_HIP(hipStreamSynchronize(s));
    g->bytes = (sizeof(int32_t) + sizeof(uint4)) * nnz + sizeof(uint2) * n + sizeof(int32_t) * (n + g->n_active) +
               sizeof(int64_t) * (g->n_active + 1) +
               (g->weighted ? sizeof(double) * (2 * nnz + n) : 0) +
               (g->n_hubs > 0 ? (sizeof(uint32_t) + sizeof(uint8_t)) * n + sizeof(int32_t) * kMaxHubs : 0) +
               (g->n_whubs > 0 ? (sizeof(uint32_t) * kWideWords + sizeof(uint16_t)) * n + sizeof(int32_t) * g->n_whubs
                               : 0);
    // The diagonal walk chooses the wide hub sums per call where the graph
    // has wide hubs and is past the size at which the ROW layout pays.
    if (g->n_whubs > 0 && g->tuning.diag_sampler != MCMF_SAMPLER_ROW)
        g->tuning.diag_sampler = MCMF_SAMPLER_AUTO;
    // Weighted rows walk by the alias method: one 16-byte record per step
    // instead of a binary search (4.6x faster diagonal walks and 3.6x faster
    // action walks on a weighted R-MAT 20).  A graph whose records do not fit
    // keeps the running sums.
    if (g->weighted) {
        const Status st = ensure_alias(g);
        if (!st)
            g->tuning.action_sampler = g->tuning.diag_sampler = MCMF_SAMPLER_ALIAS;
        else if (st.code == MCMF_E_NOMEM)
            clear_error();
        else
            return st;
    }
    return {};
}

// Walker's alias tables of the weighted rows by Vose's construction, one
// thread per row: q_j = (|a_j| d) / rowabs; "small" (q < 1) and "large"
// stacks pushed in ascending j (small grows up from stack[b], large down
// from stack[b + d - 1]: together they never hold more than d entries);
// pair the tops, give the small one prob q_s and the large one as alias,
// q_g = (q_g + q_s) - 1 back onto its stack; leftovers get prob 1 and
// themselves.  A row of zeros gets prob 1 everywhere.  The records carry
// both candidates' columns and signs, so a step needs one load.
__global__ void k_build_alias(const uint2 *node, const int32_t *col, const double *val, const double *rowabs,
                              int64_t n, uint32_t *stack, double *q, uint4 *rec) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const uint2 r = node[i];
        const uint32_t d = r.y;
        const int64_t b = r.x;
        const double W = rowabs[i];
        auto tag = [&](uint32_t j) -> uint32_t {
            return static_cast<uint32_t>(col[b + j]) | (val[b + j] < 0.0 ? 0x80000000u : 0u);
        };
        auto put = [&](uint32_t j, uint32_t a, double prob) {
            const uint64_t bits = static_cast<uint64_t>(__double_as_longlong(prob));
            rec[b + j] = make_uint4(tag(j), tag(a), static_cast<uint32_t>(bits), static_cast<uint32_t>(bits >> 32));
        };
        if (!(W > 0.0)) {
            for (uint32_t j = 0; j < d; ++j)
                put(j, j, 1.0);
            continue;
        }
        uint32_t ns = 0, nl = 0;
        for (uint32_t j = 0; j < d; ++j) {
            const double qj = (fabs(val[b + j]) * static_cast<double>(d)) / W;
            q[b + j] = qj;
            if (qj < 1.0)
                stack[b + ns++] = j;
            else
                stack[b + d - 1 - nl++] = j;
        }
        while (ns > 0 && nl > 0) {
            const uint32_t s = stack[b + --ns];
            const uint32_t big = stack[b + d - nl];
            --nl;
            const double qs = q[b + s];
            put(s, big, qs);
            const double qb = (q[b + big] + qs) - 1.0;
            q[b + big] = qb;
            if (qb < 1.0)
                stack[b + ns++] = big;
            else
                stack[b + d - 1 - nl++] = big;
        }
        while (nl > 0) {
            const uint32_t big = stack[b + d - nl];
            --nl;
            put(big, big, 1.0);
        }
        while (ns > 0) {
            const uint32_t s = stack[b + --ns];
            put(s, s, 1.0);
        }
    }
}

} // namespace

Status ensure_alias(mcmf_graph *g) {
    if (!g->weighted || g->alias_rec || g->nnz == 0)
        return {};
    // Test hook: the alias records "do not fit" (MCMF_TEST_FAIL_ALIAS=1).
    const char *no_room = getenv("MCMF_TEST_FAIL_ALIAS");
    if (no_room && no_room[0] == '1')
        return fail(MCMF_E_NOMEM, "alias records refused (MCMF_TEST_FAIL_ALIAS)");
    MCMF_HIP(hipSetDevice(g->device));
    hipStream_t s = g->stream;
    uint4 *rec = nullptr;
    MCMF_TRY(dev_alloc_sync(reinterpret_cast<void **>(&rec), sizeof(uint4) * g->nnz));
    DevBuf<uint32_t> stack;
    DevBuf<double> q;
    Status st = stack.alloc(g->nnz, s);
    if (!st)
        st = q.alloc(g->nnz, s);
    if (!st) {
        hipLaunchKernelGGL(k_build_alias, dim3(grid_for(g->n)), dim3(kThreads), 0, s, g->node, g->col, g->val,
                           g->rowabs, g->n, stack.ptr, q.ptr, rec);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            st = fail(MCMF_E_DEVICE, "alias table build: %s", hipGetErrorString(e));
    }
    if (!st) {
        const hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            st = fail(MCMF_E_DEVICE, "alias table build: %s", hipGetErrorString(e));
    }
    if (st) {
        dev_free_sync(rec, sizeof(uint4) * g->nnz);
        return st;
    }
    g->alias_rec = rec;
    g->bytes += sizeof(uint4) * g->nnz;
    return {};
}

bool auto_wide(const mcmf_graph *g, int64_t n_walks, int K) {
    if (g->n_whubs == 0 || g->weighted || K < 2 || n_walks < 1 || g->n_active == 0)
        return false;
    const int32_t act = active_wide_hubs(g, n_walks, K);
    const int32_t narrow = std::min<int32_t>(act, g->n_hubs); // summed by the EDGE walk too
    const double saved = g->whub_sq_prefix[static_cast<size_t>(act)] - g->whub_sq_prefix[static_cast<size_t>(narrow)];
    const double states = static_cast<double>(g->n_active) * static_cast<double>(n_walks) * (K - 1);
    return saved >= kWideMinSavedPerState * states;
}

int32_t active_wide_hubs(const mcmf_graph *g, int64_t n_walks, int K) {
    if (g->n_whubs == 0)
        return 0;
    int64_t min_deg = g->tuning.hub_min_degree;
    if (min_deg <= 0)
        min_deg = std::max<int64_t>(1, n_walks * (K - 1) / 4);
    int32_t c = 0; // wide hubs are sorted by degree: the active ones are a prefix
    while (c < g->n_whubs && g->whub_deg_host[static_cast<size_t>(c)] >= min_deg)
        ++c;
    return c;
}

uint32_t active_hubs(const mcmf_graph *g, int64_t n_walks, int K) {
    if (g->n_hubs == 0)
        return 0u;
    int64_t min_deg = g->tuning.hub_min_degree;
    if (min_deg <= 0)
        min_deg = std::max<int64_t>(1, n_walks * (K - 1) / 4);
    uint32_t m = 0u;
    for (int h = 0; h < g->n_hubs; ++h)
        if (g->hub_deg_host[h] >= min_deg)
            m |= 1u << h;
    return m;
}

Status fill_u8(uint8_t *out, uint8_t value, int64_t n, hipStream_t s) { return fill_impl(out, value, n, s); }
Status fill_i32(int32_t *out, int32_t value, int64_t n, hipStream_t s) { return fill_impl(out, value, n, s); }
Status fill_f64(double *out, double value, int64_t n, hipStream_t s) { return fill_impl(out, value, n, s); }
Status fill_u64(uint64_t *out, uint64_t value, int64_t n, hipStream_t s) { return fill_impl(out, value, n, s); }

Status compact(const uint8_t *flags, int64_t n, uint8_t match, int32_t *out, int64_t *count,
               hipStream_t s) {
    *count = 0;
    if (n <= 0)
        return {};
    const int64_t nb = (n + kCompactSpan - 1) / kCompactSpan;
    DevBuf<uint32_t> counts;
    DevBuf<unsigned long long> total;
    MCMF_TRY(counts.alloc(nb, s));
    MCMF_TRY(total.alloc(1, s));
    hipLaunchKernelGGL(k_compact_count, dim3(nb), dim3(kThreads), 0, s, flags, n, match, counts.ptr);
    MCMF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, s, counts.ptr, nb, total.ptr);
    MCMF_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_compact_write, dim3(nb), dim3(kThreads), 0, s, flags, n, match, counts.ptr,
                       out);
    MCMF_HIP(hipGetLastError());
    unsigned long long c = 0;
    MCMF_HIP(hipMemcpyAsync(&c, total.ptr, sizeof c, hipMemcpyDeviceToHost, s));
    MCMF_HIP(hipStreamSynchronize(s));
    *count = static_cast<int64_t>(c);
    return {};
}

// B = [[0, A], [A^T, 0]] of a directed graph A, on the host: rows i < n are
// A's rows with columns shifted by n; row n + j lists the rows i with
// a_ij != 0 in ascending order (a counting sort over A's rows taken in order
// is stable, so no sort is needed).
Status digraph_symmetrize(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          std::vector<int64_t> &b_ptr, std::vector<int32_t> &b_col,
                          std::vector<double> &b_val) {
    if (n >= (int64_t(1) << 30))
        return fail(MCMF_E_UNSUPPORTED, "MCMF_DIGRAPH needs n < 2^30 (got %lld)", static_cast<long long>(n));
    std::vector<int64_t> hptr;
    std::vector<int32_t> hcol;
    std::vector<double> hval;
    const int64_t *rp = row_ptr;
    if (classify(row_ptr) == Mem::Device) {
        hptr.resize(static_cast<size_t>(n + 1));
        MCMF_HIP(hipMemcpy(hptr.data(), row_ptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
        rp = hptr.data();
    }
    if (rp[0] != 0)
        return fail(MCMF_E_CSR, "row_ptr[0] = %lld, expected 0", static_cast<long long>(rp[0]));
    for (int64_t i = 0; i < n; ++i)
        if (rp[i + 1] < rp[i])
            return fail(MCMF_E_CSR, "row_ptr decreases at row %lld", static_cast<long long>(i));
    const int64_t nnz = rp[n];
    if (2 * nnz >= (int64_t(1) << 32))
        return fail(MCMF_E_UNSUPPORTED, "MCMF_DIGRAPH needs 2 nnz < 2^32 (nnz = %lld)",
                    static_cast<long long>(nnz));
    if (nnz > 0 && !col)
        return fail(MCMF_E_ARG, "col_idx is NULL with nnz = %lld", static_cast<long long>(nnz));
    const int32_t *cp = col;
    if (nnz > 0 && classify(col) == Mem::Device) {
        hcol.resize(static_cast<size_t>(nnz));
        MCMF_HIP(hipMemcpy(hcol.data(), col, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
        cp = hcol.data();
    }
    const double *vp = val;
    if (val && nnz > 0 && classify(val) == Mem::Device) {
        hval.resize(static_cast<size_t>(nnz));
        MCMF_HIP(hipMemcpy(hval.data(), val, sizeof(double) * nnz, hipMemcpyDeviceToHost));
        vp = hval.data();
    }
    for (int64_t e = 0; e < nnz; ++e)
        if (cp[e] < 0 || cp[e] >= n)
            return fail(MCMF_E_CSR, "col_idx[%lld] = %d outside [0, %lld)", static_cast<long long>(e), cp[e],
                        static_cast<long long>(n));
    b_ptr.assign(static_cast<size_t>(2 * n + 1), 0);
    b_col.resize(static_cast<size_t>(2 * nnz));
    if (vp)
        b_val.resize(static_cast<size_t>(2 * nnz));
    for (int64_t i = 0; i < n; ++i)
        b_ptr[i + 1] = rp[i + 1];
    for (int64_t e = 0; e < nnz; ++e)
        ++b_ptr[n + cp[e] + 1];
    for (int64_t j = n; j < 2 * n; ++j)
        b_ptr[j + 1] += b_ptr[j];
    for (int64_t e = 0; e < nnz; ++e) {
        b_col[e] = static_cast<int32_t>(cp[e] + n);
        if (vp)
            b_val[e] = vp[e];
    }
    std::vector<int64_t> cursor(b_ptr.begin() + n, b_ptr.begin() + 2 * n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int64_t pos = cursor[cp[e]]++;
            b_col[pos] = static_cast<int32_t>(i);
            if (vp)
                b_val[pos] = vp[e];
        }
    return {};
}

} // namespace mcmf

using namespace mcmf;

extern "C" mcmf_status mcmf_graph_create(int64_t n, const int64_t *row_ptr, const int32_t *col_idx,
                                         const double *values, uint32_t flags, mcmf_graph **out) {
    clear_error();
    if (!out) {
        fail(MCMF_E_ARG, "out is NULL");
        return MCMF_E_ARG;
    }
    if (n < 0 || n >= (int64_t(1) << 31)) {
        fail(MCMF_E_ARG, "n = %lld outside [0, 2^31)", static_cast<long long>(n));
        return MCMF_E_ARG;
    }
    if (!row_ptr) {
        fail(MCMF_E_ARG, "row_ptr is NULL");
        return MCMF_E_ARG;
    }
    const uint32_t known = MCMF_SYMMETRIC | MCMF_VALIDATE | MCMF_DIGRAPH;
    if (flags & ~known) {
        fail(MCMF_E_ARG, "unknown flag bits 0x%x", flags & ~known);
        return MCMF_E_ARG;
    }
    if ((flags & MCMF_DIGRAPH) && (flags & MCMF_SYMMETRIC)) {
        fail(MCMF_E_ARG, "MCMF_DIGRAPH and MCMF_SYMMETRIC exclude each other (B is symmetric by construction)");
        return MCMF_E_ARG;
    }
    std::vector<int64_t> b_ptr;
    std::vector<int32_t> b_col;
    std::vector<double> b_val;
    if (flags & MCMF_DIGRAPH) {
        Status st = digraph_symmetrize(n, row_ptr, col_idx, values, b_ptr, b_col, b_val);
        if (st)
            return st.code;
        n = 2 * n;
        row_ptr = b_ptr.data();
        col_idx = b_col.data();
        values = values ? b_val.data() : nullptr;
        flags = (flags & MCMF_VALIDATE) | MCMF_SYMMETRIC;
    }
    mcmf_graph *g = new (std::nothrow) mcmf_graph();
    if (!g) {
        fail(MCMF_E_NOMEM, "host allocation failed");
        return MCMF_E_NOMEM;
    }
    Status st = build_graph(g, n, row_ptr, col_idx, values, flags);
    if (st) {
        const std::string msg = mcmf_last_error();
        free_graph(g);
        set_error("%s", msg.c_str());
        return st.code;
    }
    *out = g;
    return MCMF_OK;
}

extern "C" void mcmf_graph_destroy(mcmf_graph *g) { free_graph(g); }

extern "C" mcmf_status mcmf_graph_info(const mcmf_graph *g, int64_t *n, int64_t *nnz, int64_t *d_max,
                                       int64_t *active_rows) {
    clear_error();
    if (!g) {
        fail(MCMF_E_ARG, "graph is NULL");
        return MCMF_E_ARG;
    }
    if (n)
        *n = g->n;
    if (nnz)
        *nnz = g->nnz;
    if (d_max)
        *d_max = g->d_max;
    if (active_rows)
        *active_rows = g->n_active;
    return MCMF_OK;
}
