// Host-side plumbing shared by the library's translation units: error state,
// status propagation, device-memory accounting and pointer classification.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "mcmf.h"

namespace mcmf {

// Thread-local message behind mcmf_last_error().
void set_error(const char *fmt, ...) __attribute__((format(printf, 1, 2)));
void clear_error();

// A status plus the place it came from; MCMF_OK converts to false.
struct Status {
    mcmf_status code = MCMF_OK;
    explicit operator bool() const { return code != MCMF_OK; }
};

Status fail(mcmf_status code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
Status hip_fail(hipError_t e, const char *what, const char *file, int line);

#define MCMF_HIP(expr)                                                        \
    do {                                                                      \
        hipError_t e_ = (expr);                                               \
        if (e_ != hipSuccess)                                                 \
            return ::mcmf::hip_fail(e_, #expr, __FILE__, __LINE__);           \
    } while (0)

#define MCMF_TRY(expr)                                                        \
    do {                                                                      \
        ::mcmf::Status s_ = (expr);                                           \
        if (s_)                                                               \
            return s_;                                                        \
    } while (0)

// Where a caller pointer lives.
enum class Mem { Host, Device };
Mem classify(const void *p);

// Device memory accounting against an optional byte budget (environment
// variable MCMF_HBM_BUDGET_BYTES).  MCMF_TEST_FAIL_ALLOC=1 makes every
// allocation fail, MCMF_TEST_FAIL_ALLOC_ABOVE=B every one of more than B
// bytes, so the out-of-memory paths can be exercised on purpose.
Status dev_alloc(void **p, size_t bytes, hipStream_t stream);
void dev_free(void *p, size_t bytes, hipStream_t stream);
Status dev_alloc_sync(void **p, size_t bytes);
void dev_free_sync(void *p, size_t bytes);

// Temporary device buffer that is released on scope exit, stream ordered.
template <class T>
struct DevBuf {
    T *ptr = nullptr;
    size_t count = 0;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { reset(); }
    Status alloc(size_t n, hipStream_t s) {
        reset();
        stream = s;
        count = n;
        if (n == 0)
            return {};
        Status st = dev_alloc(reinterpret_cast<void **>(&ptr), n * sizeof(T), s);
        if (st) {
            ptr = nullptr;
            count = 0;
        }
        return st;
    }
    void reset() {
        if (ptr)
            dev_free(ptr, count * sizeof(T), stream);
        ptr = nullptr;
        count = 0;
    }
};

// Device view of a caller array: the array itself or a staged copy.
template <class T>
struct View {
    T *ptr = nullptr;
    DevBuf<T> staged;
    bool host = false;
    Status in(const T *p, size_t count, hipStream_t s) {
        host = classify(p) == Mem::Host;
        if (!host) {
            ptr = const_cast<T *>(p);
            return {};
        }
        MCMF_TRY(staged.alloc(count, s));
        ptr = staged.ptr;
        if (count)
            MCMF_HIP(hipMemcpyAsync(ptr, p, sizeof(T) * count, hipMemcpyHostToDevice, s));
        return {};
    }
    Status out(T *p, size_t count, hipStream_t s) {
        host = classify(p) == Mem::Host;
        if (!host) {
            ptr = p;
            return {};
        }
        MCMF_TRY(staged.alloc(count, s));
        ptr = staged.ptr;
        return {};
    }
    Status copy_back(T *p, size_t count, hipStream_t s) {
        if (host && count)
            MCMF_HIP(hipMemcpyAsync(p, ptr, sizeof(T) * count, hipMemcpyDeviceToHost, s));
        return {};
    }
};

// Coefficients c_0..c_K of the function family (host, FP64, in sequence).
Status make_coeffs(const mcmf_fn *f, int K, double *c);

int num_cus();

// Entries of a gather launch's item map for `rows` distinct start rows of a
// graph with nnz stored entries and rows of at most d_max entries, cut into
// items of `item` neighbours: the items there can be, at most kMaxItemMap
// (items beyond take the binary-search path).
constexpr int64_t kMaxItemMap = int64_t(1) << 23;
int64_t item_map_entries(int64_t rows, int64_t nnz, int64_t d_max, uint32_t item);

// Test hook: MCMF_TEST_ITEM_MAP_CAP=C caps the gather launches' item maps at
// C entries, so that the items beyond take the binary-search path; returns
// cap unchanged without it.
int64_t item_map_cap(int64_t cap);

// Default size of a call's diagonal visit-record buffer: the
// MCMF_DIAG_CHUNK_BYTES environment value, else 1/16 of device memory
// clamped to [256 MiB, 16 GiB] (fewer, larger chunks mean fewer launch tails;
// at most half the block cache's 1/8 of device memory, so the buffer stays
// cached between calls).  Without the environment value a call that cannot
// get its buffer halves it, down to kMinVisitChunkBytes.
constexpr int64_t kMinVisitChunkBytes = int64_t(256) << 20;
int64_t default_visit_chunk_bytes();
bool visit_chunk_bytes_fixed();

// Total memory of the current device (cached; 64 GiB if it cannot be read).
uint64_t device_memory_bytes();

// Neighbours per diagonal-gather work item when the tuning leaves it open.
constexpr int32_t kDefaultGatherItem = 256;

// Hub rows of the diagonal gather: at most one per bit of a 32-bit mask.
constexpr int kMaxHubs = 32;
constexpr uint8_t kNoHub = 0xFF;

// Wide hubs: up to kMaxWideHubs hub rows, with a 128-byte mask per node
// (kWideWords words, one 128-byte line) of the wide hubs adjacent to it.
constexpr int kWideWords = 32;
constexpr int kMaxWideHubs = 32 * kWideWords; // 1024
constexpr uint16_t kNoWideHub = 0xFFFF;
// MCMF_SAMPLER_AUTO takes the wide hub sums when they save at least this
// many probed column entries per recorded walk state.
constexpr double kWideMinSavedPerState = 4.0;

} // namespace mcmf

// Opaque graph handle: the device copy of A and its per-row metadata.
struct mcmf_graph {
    int device = 0;
    int64_t n = 0;
    int64_t nnz = 0;
    int64_t d_max = 0;
    int64_t n_active = 0; // rows with at least one entry
    bool weighted = false;
    bool symmetric = false;
    hipStream_t stream = nullptr; // the graph's own stream

    // Device arrays.
    int64_t *row_ptr = nullptr; // [n+1]
    int32_t *col = nullptr;     // [nnz]
    double *val = nullptr;      // [nnz] or null
    double *rowabs = nullptr;   // [n] sum |a| (weighted only)
    double *cum = nullptr;      // [nnz] running sums of |a| per row (weighted only)
    // [nnz] alias records of weighted rows, built on first use of
    // MCMF_SAMPLER_ALIAS: {col_j | sign_j << 31, col_a | sign_a << 31,
    // prob_j low word, high word} with a = alias_j (sign: a < 0).
    uint4 *alias_rec = nullptr;
    uint2 *node = nullptr;      // [n] {first entry, row length}
    // [nnz] per stored entry a_ij: {j, first entry of row j, length of row j,
    // hubmask[j] (0 without hubs)}.  A walk step then needs one dependent
    // load: the entry it picks already carries the record of the row it
    // moves to.
    uint4 *edge = nullptr;
    int32_t *active = nullptr;  // [n_active] rows with entries, ascending
    // [n_active + 1] first diagonal-gather work item of each active row
    // (exclusive prefix sums of ceil(row length / 256)).
    int64_t *active_items = nullptr;
    // Rows grouped by length for the sparse products: short (<= 64 entries,
    // including empty rows), medium (<= 4096), long.
    int32_t *bin_rows = nullptr; // [n] concatenated bins
    int64_t bin_count[3] = {0, 0, 0};
    int64_t bin_offset[3] = {0, 0, 0};
    size_t bytes = 0;
    // Walk-kernel choices (mcmf_graph_set_tuning / mcmf_tune).
    mcmf_tuning tuning = {MCMF_SAMPLER_VALUE, 0, MCMF_SAMPLER_EDGE, 0, {0, 0, 0, 0}, {0, 0, 0, 0}, 0, 0, 0, {0, 0},
                          0, 0, {0, 0, 0}, {0, 0, 0, 0}, {0, 0}, 0, {0, 0}, 0, 0};
    // Hub rows (unweighted symmetric graphs with strictly increasing rows):
    // the rows of largest degree, at most kMaxHubs.  hubmask[j] has bit h set
    // when j is a column of row hub_rows[h] (by symmetry: when j is adjacent
    // to hub h); hub_of[i] = h for hub row i, kNoHub elsewhere.
    bool strict_rows = false;
    int32_t n_hubs = 0;
    int32_t hub_rows_host[mcmf::kMaxHubs] = {};
    int64_t hub_deg_host[mcmf::kMaxHubs] = {};
    int32_t *hub_rows = nullptr; // [kMaxHubs]
    uint32_t *hubmask = nullptr; // [n]
    uint8_t *hub_of = nullptr;   // [n]
    // Q_k table overflows (lost inserts) of asynchronous diagonal calls on
    // this graph; checked and cleared by its next synchronising call.
    unsigned long long *async_overflow = nullptr; // [1]
    // Wide hubs (unweighted symmetric graphs with strictly increasing rows
    // and more than kMaxHubs rows with entries): the up to kMaxWideHubs rows
    // of largest degree (the first kMaxHubs are hub_rows), degree descending;
    // whub_of[i] = wide hub index of row i, kNoWideHub elsewhere;
    // wmask[i * kWideWords + w] = bits of the wide hubs 32w..32w+31 adjacent
    // to i (128 bytes per node, line aligned).
    int32_t n_whubs = 0;
    std::vector<int64_t> whub_deg_host;
    std::vector<double> whub_sq_prefix; // [n_whubs + 1] prefix sums of deg^2 (MCMF_SAMPLER_AUTO)
    int32_t *whub_rows = nullptr; // [n_whubs]
    uint16_t *whub_of = nullptr;  // [n]
    uint32_t *wmask = nullptr;    // [n * kWideWords]
};
