// mcmf_action_noalloc: RandFunmAction (Section 3.4, Algorithm 3) for callers
// that cannot allocate device memory.  The call's temporaries live in one
// file-scope device array, `scratch`, instead of per-call allocations:
//
//   [0, 32760)          c_{t+2}, t = 0..K-2 (at most 4095 FP64 values)
//   [32768, +8n)        r = s A v
//   [32768 + 8n, +8n)   q_k of the walks
//
// The walks read the graph's edge or row records (never the per-call value
// records, which would need 16 bytes per stored entry), so the walks, and
// the estimate, are those of mcmf_action on the same arguments.
#include <mutex>

#include "ops.hpp"

namespace mcmf {

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kCoefBytes = 32768;
constexpr int kMaxDevices = 64;

// One copy per device; host code reaches it only through the address that
// hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array, looked up once per device.
Status scratch_on(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices)
        return fail(MCMF_E_UNSUPPORTED, "device %d beyond the %d devices the no-allocation path serves",
                    device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        MCMF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p)
            return fail(MCMF_E_DEVICE, "hipGetSymbolAddress returned a null scratch address");
        g_scratch_ptr[device] = p;
    }
    *out = static_cast<unsigned char *>(g_scratch_ptr[device]);
    return {};
}

Status run_action_noalloc(const mcmf_graph *g, const mcmf_fn *f, const double *v, int64_t N, int32_t K,
                          const mcmf_opts *o, double *out) {
    MCMF_TRY(check_common(g, f, N, K, o));
    if (!v || !out)
        return fail(MCMF_E_ARG, "v and out must not be NULL");
    if (v == out)
        return fail(MCMF_E_ARG, "out may not alias v");
    if (g->n > MCMF_NOALLOC_MAX_ROWS)
        return fail(MCMF_E_UNSUPPORTED, "n = %lld exceeds the no-allocation limit of %lld rows",
                    static_cast<long long>(g->n), static_cast<long long>(MCMF_NOALLOC_MAX_ROWS));
    if (o && o->allocation != MCMF_ALLOC_PER_ROW)
        return fail(MCMF_E_UNSUPPORTED, "mcmf_action_noalloc runs MCMF_ALLOC_PER_ROW only");
    if (o && o->walks_out)
        return fail(MCMF_E_UNSUPPORTED, "mcmf_action_noalloc does not write walks_out");
    static_assert(kCoefBytes >= sizeof(double) * 4095, "coefficient area");
    static_assert(kCoefBytes + sizeof(double) * 2 * MCMF_NOALLOC_MAX_ROWS <= kScratchBytes, "scratch size");
    MCMF_HIP(hipSetDevice(g->device));
    if (classify(v) != Mem::Device || classify(out) != Mem::Device)
        return fail(MCMF_E_ARG, "mcmf_action_noalloc needs v and out in device memory");
    uint64_t *digest = o ? o->path_digest : nullptr;
    double *q_out = o ? o->q_out : nullptr;
    if ((digest && classify(digest) != Mem::Device) || (q_out && classify(q_out) != Mem::Device))
        return fail(MCMF_E_ARG, "mcmf_action_noalloc needs path_digest and q_out in device memory");
    double c[4097];
    MCMF_TRY(make_coeffs(f, K, c));
    unsigned char *base = nullptr;
    MCMF_TRY(scratch_on(g->device, &base));
    hipStream_t s = (o && o->stream) ? static_cast<hipStream_t>(o->stream) : g->stream;
    const int64_t n = g->n;
    double *coef = reinterpret_cast<double *>(base);
    double *r = reinterpret_cast<double *>(base + kCoefBytes);
    double *q = r + n;

    if (digest)
        MCMF_TRY(fill_u64(digest, 0, n, s));
    MCMF_TRY(spmv_r(g, v, f->scale, r, s));
    if (K >= 2) {
        // Pageable source: the copy has taken the values when it returns.
        MCMF_HIP(hipMemcpyAsync(coef, c + 2, sizeof(double) * (K - 1), hipMemcpyHostToDevice, s));
        // Every q entry is written: zeros first, then q_k of each start row.
        MCMF_TRY(fill_f64(q, 0.0, n, s));
        WalkParams p = walk_params(o, coef, K, f->scale, N);
        const int sampler = g->tuning.action_sampler;
        p.sampler = sampler == MCMF_SAMPLER_VALUE ? MCMF_SAMPLER_EDGE : sampler;
        MCMF_TRY(action_walks(g, r, g->active, g->n_active, p, q, digest, nullptr, s));
    }
    MCMF_TRY(spmv_assemble(g, v, r, K >= 2 ? q : nullptr, c[0], K >= 1 ? c[1] : 0.0, f->scale, out, s));
    if (q_out) {
        if (K >= 2 && n)
            MCMF_HIP(hipMemcpyAsync(q_out, q, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        else
            MCMF_TRY(fill_f64(q_out, 0.0, n, s));
    }
    if (!(o && o->stream))
        MCMF_HIP(hipStreamSynchronize(s));
    return {};
}

} // namespace

} // namespace mcmf

extern "C" mcmf_status mcmf_action_noalloc(const mcmf_graph *g, const mcmf_fn *f, const double *v,
                                           int64_t n_walks, int32_t K, const mcmf_opts *opts,
                                           double *out) {
    mcmf::clear_error();
    return mcmf::run_action_noalloc(g, f, v, n_walks, K, opts, out).code;
}
