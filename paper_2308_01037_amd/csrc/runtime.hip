// Error state, device-memory accounting, pointer classification and the
// function-coefficient tables.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#include "common.hpp"

namespace mcmf {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

Status fail(mcmf_status code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    Status s;
    s.code = code;
    return s;
}

Status hip_fail(hipError_t e, const char *what, const char *file, int line) {
    const char *base = strrchr(file, '/');
    Status s = fail(e == hipErrorOutOfMemory ? MCMF_E_NOMEM : MCMF_E_DEVICE, "%s failed: %s (%s:%d)",
                    what, hipGetErrorString(e), base ? base + 1 : file, line);
    (void)hipGetLastError();
    return s;
}

Mem classify(const void *p) {
    if (!p)
        return Mem::Host;
    hipPointerAttribute_t attr;
    memset(&attr, 0, sizeof attr);
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return Mem::Host;
    }
    return (attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged) ? Mem::Device
                                                                                 : Mem::Host;
}

// ---------------------------------------------------------------- memory

static std::atomic<int64_t> g_bytes_in_use{0};

static int64_t budget_bytes() {
    static int64_t budget = [] {
        const char *s = getenv("MCMF_HBM_BUDGET_BYTES");
        return s ? static_cast<int64_t>(strtoll(s, nullptr, 10)) : int64_t(0);
    }();
    return budget;
}

// Test hooks: MCMF_TEST_FAIL_ALLOC=1 refuses every allocation,
// MCMF_TEST_FAIL_ALLOC_ABOVE=B every allocation of more than B bytes.
static bool forced_failure(size_t bytes) {
    const char *s = getenv("MCMF_TEST_FAIL_ALLOC");
    if (s && s[0] == '1')
        return true;
    const char *a = getenv("MCMF_TEST_FAIL_ALLOC_ABOVE");
    return a && a[0] && bytes > static_cast<size_t>(strtoull(a, nullptr, 10));
}

static Status reserve(size_t bytes) {
    if (forced_failure(bytes))
        return fail(MCMF_E_NOMEM, "device allocation of %zu bytes refused (MCMF_TEST_FAIL_ALLOC)",
                    bytes);
    const int64_t b = budget_bytes();
    const int64_t now = g_bytes_in_use.fetch_add(static_cast<int64_t>(bytes)) + static_cast<int64_t>(bytes);
    if (b > 0 && now > b) {
        g_bytes_in_use.fetch_sub(static_cast<int64_t>(bytes));
        return fail(MCMF_E_NOMEM, "device byte budget exceeded: %lld in use + %zu requested > %lld",
                    static_cast<long long>(now - static_cast<int64_t>(bytes)), bytes,
                    static_cast<long long>(b));
    }
    return {};
}

static void unreserve(size_t bytes) { g_bytes_in_use.fetch_sub(static_cast<int64_t>(bytes)); }

// Block cache for the per-call temporaries.  Freed blocks stay with the
// library (grouped by size class, at most 1/8 over the request) and are
// handed out again: to the same stream at once (stream order protects the
// reuse), to another stream once an event recorded at the free has passed.
// Device memory is only returned to the driver when the cache grows past
// its limit or an allocation fails, so a steady stream of calls maps no new
// memory.
namespace {

struct CachedBlock {
    void *p;
    size_t bytes;
    int device;
    hipStream_t stream;
    hipEvent_t freed;
};

std::mutex g_cache_mu;
std::vector<CachedBlock> g_cache;
std::vector<hipEvent_t> g_spare_events;
size_t g_cached_bytes = 0;

size_t cache_limit() {
    static size_t limit = [] {
        const char *s = getenv("MCMF_CACHE_BYTES");
        if (s)
            return static_cast<size_t>(strtoull(s, nullptr, 10));
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            return size_t(8) << 30;
        }
        return total_b / 8;
    }();
    return limit;
}

// Size classes: 8 per power of two, at least 4 KiB.
size_t size_class(size_t bytes) {
    if (bytes <= 4096)
        return 4096;
    const int top = 63 - __builtin_clzll(static_cast<unsigned long long>(bytes - 1));
    const size_t step = size_t(1) << (top >= 3 ? top - 3 : 0);
    return (bytes + step - 1) / step * step;
}

// Frees cached blocks (oldest first) until at most `keep` bytes stay cached.
// The caller holds g_cache_mu.
void trim_locked(size_t keep) {
    while (g_cached_bytes > keep && !g_cache.empty()) {
        const CachedBlock b = g_cache.front();
        g_cache.erase(g_cache.begin());
        g_cached_bytes -= b.bytes;
        int cur = 0;
        (void)hipGetDevice(&cur);
        (void)hipSetDevice(b.device);
        (void)hipEventSynchronize(b.freed);
        (void)hipFree(b.p);
        (void)hipSetDevice(cur);
        g_spare_events.push_back(b.freed);
    }
}

} // namespace

Status dev_alloc(void **p, size_t bytes, hipStream_t stream) {
    *p = nullptr;
    if (bytes == 0)
        return {};
    const size_t cls = size_class(bytes);
    MCMF_TRY(reserve(cls));
    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e != hipSuccess) {
        unreserve(cls);
        return hip_fail(e, "hipGetDevice", __FILE__, __LINE__);
    }
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        for (size_t i = 0; i < g_cache.size(); ++i) {
            CachedBlock &b = g_cache[i];
            if (b.device != device || b.bytes != cls)
                continue;
            bool ready = b.stream == stream;
            if (!ready) {
                const hipError_t q = hipEventQuery(b.freed);
                ready = q == hipSuccess;
                if (q != hipSuccess)
                    (void)hipGetLastError();
            }
            if (!ready)
                continue;
            *p = b.p;
            g_cached_bytes -= b.bytes;
            g_spare_events.push_back(b.freed);
            g_cache.erase(g_cache.begin() + static_cast<std::ptrdiff_t>(i));
            return {};
        }
    }
    e = hipMalloc(p, cls);
    if (e == hipErrorOutOfMemory) {
        (void)hipGetLastError();
        {
            std::lock_guard<std::mutex> lock(g_cache_mu);
            trim_locked(0);
        }
        e = hipMalloc(p, cls);
    }
    if (e != hipSuccess) {
        unreserve(cls);
        *p = nullptr;
        return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    }
    return {};
}

void dev_free(void *p, size_t bytes, hipStream_t stream) {
    if (!p)
        return;
    const size_t cls = size_class(bytes);
    unreserve(cls);
    int device = 0;
    (void)hipGetDevice(&device);
    std::lock_guard<std::mutex> lock(g_cache_mu);
    hipEvent_t ev = nullptr;
    if (!g_spare_events.empty()) {
        ev = g_spare_events.back();
        g_spare_events.pop_back();
    } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        ev = nullptr;
    }
    if (!ev || hipEventRecord(ev, stream) != hipSuccess) {
        // No event to order a reuse by: give the block back to the driver.
        (void)hipGetLastError();
        if (ev)
            g_spare_events.push_back(ev);
        (void)hipStreamSynchronize(stream);
        (void)hipFree(p);
        return;
    }
    g_cache.push_back(CachedBlock{p, cls, device, stream, ev});
    g_cached_bytes += cls;
    if (g_cached_bytes > cache_limit())
        trim_locked(cache_limit());
}

Status dev_alloc_sync(void **p, size_t bytes) {
    *p = nullptr;
    if (bytes == 0)
        return {};
    MCMF_TRY(reserve(bytes));
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        unreserve(bytes);
        *p = nullptr;
        return hip_fail(e, "hipMalloc", __FILE__, __LINE__);
    }
    return {};
}

void dev_free_sync(void *p, size_t bytes) {
    if (!p)
        return;
    (void)hipFree(p);
    unreserve(bytes);
}

// ---------------------------------------------------------------- coefficients

Status make_coeffs(const mcmf_fn *f, int K, double *c) {
    switch (f->kind) {
    case MCMF_FN_EXP:
        c[0] = 1.0;
        for (int k = 1; k <= K; ++k)
            c[k] = c[k - 1] / static_cast<double>(k);
        return {};
    case MCMF_FN_RESOLVENT:
        for (int k = 0; k <= K; ++k)
            c[k] = 1.0;
        return {};
    case MCMF_FN_COEFFS:
        if (!f->coeffs)
            return fail(MCMF_E_ARG, "MCMF_FN_COEFFS needs a coefficient array");
        if (f->n_coeffs < K + 1)
            return fail(MCMF_E_ARG, "MCMF_FN_COEFFS has %d coefficients, K=%d needs %d", f->n_coeffs,
                        K, K + 1);
        if (classify(f->coeffs) != Mem::Host)
            return fail(MCMF_E_ARG, "coefficients must be in host memory");
        for (int k = 0; k <= K; ++k) {
            if (!std::isfinite(f->coeffs[k]))
                return fail(MCMF_E_ARG, "coefficient c_%d is not finite", k);
            c[k] = f->coeffs[k];
        }
        return {};
    default:
        return fail(MCMF_E_ARG, "unknown function kind %d", f->kind);
    }
}

uint64_t device_memory_bytes() {
    static uint64_t bytes = [] {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            (void)hipGetLastError();
            return uint64_t(64) << 30;
        }
        return static_cast<uint64_t>(total_b);
    }();
    return bytes;
}

int64_t item_map_entries(int64_t rows, int64_t nnz, int64_t d_max, uint32_t item) {
    const int64_t it = item > 0 ? item : 1;
    // Each row has at most ceil(d_max / item) items, and the rows together
    // one each plus one per `item` of their (at most nnz) entries.
    const int64_t per_row = (d_max + it - 1) / it;
    const int64_t by_rows = per_row > 0 && rows > kMaxItemMap / per_row ? kMaxItemMap : rows * per_row;
    const int64_t by_nnz = rows + nnz / it + 1;
    return std::min(kMaxItemMap, std::min(by_rows, by_nnz));
}

int64_t item_map_cap(int64_t cap) {
    const char *e = getenv("MCMF_TEST_ITEM_MAP_CAP");
    if (!e || !e[0])
        return cap;
    const int64_t c = strtoll(e, nullptr, 10);
    return c >= 0 && c < cap ? c : cap;
}

bool visit_chunk_bytes_fixed() { return getenv("MCMF_DIAG_CHUNK_BYTES") != nullptr; }

int64_t default_visit_chunk_bytes() {
    if (const char *e = getenv("MCMF_DIAG_CHUNK_BYTES"))
        return std::max<int64_t>(1, strtoll(e, nullptr, 10));
    return std::min<int64_t>(int64_t(16) << 30,
                             std::max<int64_t>(kMinVisitChunkBytes, static_cast<int64_t>(device_memory_bytes() / 16)));
}

int num_cus() {
    static int cus = [] {
        int dev = 0;
        hipDeviceProp_t prop;
        if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            return 256;
        }
        return prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
    }();
    return cus;
}

} // namespace mcmf

extern "C" const char *mcmf_status_string(mcmf_status s) {
    switch (s) {
    case MCMF_OK: return "MCMF_OK";
    case MCMF_E_ARG: return "MCMF_E_ARG";
    case MCMF_E_CSR: return "MCMF_E_CSR";
    case MCMF_E_NOT_SYMMETRIC: return "MCMF_E_NOT_SYMMETRIC";
    case MCMF_E_NOMEM: return "MCMF_E_NOMEM";
    case MCMF_E_DEVICE: return "MCMF_E_DEVICE";
    case MCMF_E_UNSUPPORTED: return "MCMF_E_UNSUPPORTED";
    }
    return "MCMF_E_UNKNOWN";
}

extern "C" const char *mcmf_last_error(void) { return mcmf::g_last_error.c_str(); }
