// Device-side building blocks: the counter-based random stream, the
// transition index, the path hash and wavefront/workgroup reductions.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mcmf {
namespace dev {

// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11, Section 5).  Each of
// the ten rounds multiplies word 0 by 0xD2511F53 and word 2 by 0xCD9E8D57;
// the new words are (hi2 ^ w1 ^ k0, lo2, hi0 ^ w3 ^ k1, lo0).  The key
// advances by the Weyl increments 0x9E3779B9 / 0xBB67AE85 (fractional bits
// of the golden ratio and of sqrt 3) after every round.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint32_t lo_a = 0xD2511F53u * c.x;
        const uint32_t hi_a = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo_b = 0xCD9E8D57u * c.z;
        const uint32_t hi_b = __umulhi(0xCD9E8D57u, c.z);
        c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// floor(u * deg / 2^64) for u = hi * 2^32 + lo, exact in 64-bit arithmetic:
// (hi*deg + floor(lo*deg / 2^32)) / 2^32, which cannot overflow for deg < 2^32.
__device__ __forceinline__ uint32_t uniform_index(uint32_t lo, uint32_t hi, uint32_t deg) {
    const uint64_t low_part = (static_cast<uint64_t>(lo) * deg) >> 32;
    return static_cast<uint32_t>((static_cast<uint64_t>(hi) * deg + low_part) >> 32);
}

// u53 = (u >> 11) * 2^-53 in [0, 1).
__device__ __forceinline__ double unit53(uint32_t lo, uint32_t hi) {
    const uint64_t u = (static_cast<uint64_t>(hi) << 32) | lo;
    return static_cast<double>(u >> 11) * 0x1p-53;
}

// FNV-1a over 32-bit words, for path digests.
constexpr uint64_t kFnvBasis = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;
__device__ __forceinline__ uint64_t fnv_step(uint64_t h, uint32_t word) {
    return (h ^ static_cast<uint64_t>(word)) * kFnvPrime;
}

// ---- reductions over a 64-wide wavefront ----

// A value known to be equal on every lane of the wavefront, moved to a
// scalar register so that what is computed from it stays scalar too.
__device__ __forceinline__ int32_t uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ int64_t uniform(int64_t x) {
    const uint64_t u = static_cast<uint64_t>(x);
    const uint32_t lo = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u));
    const uint32_t hi = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(u >> 32));
    return static_cast<int64_t>((uint64_t(hi) << 32) | lo);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    return x;
}

// Sum inside aligned groups of G lanes (G a power of two <= 64).
template <int G>
__device__ __forceinline__ double group_sum(double x) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    return x;
}

// Workgroup sum; every thread gets the total.  scratch holds one value per
// wavefront (blockDim.x / 64 <= 16).
template <class T>
__device__ __forceinline__ T block_sum(T x, T *scratch) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    __syncthreads();
    if (lane == 0)
        scratch[wave] = x;
    __syncthreads();
    T total = T(0);
    for (int w = 0; w < waves; ++w)
        total += scratch[w];
    return total;
}

// Exclusive prefix sum of one value per thread across the workgroup;
// *total receives the sum.  scratch: one slot per wavefront.  scratch_free:
// the caller has a barrier after the last read of scratch by an earlier scan,
// so the scan skips its own.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t x, uint32_t *scratch,
                                                         uint32_t *total, bool scratch_free = false) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int waves = (blockDim.x + 63) >> 6;
    uint32_t incl = x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += y;
    }
    if (!scratch_free) // a previous scan may still be reading scratch
        __syncthreads();
    if (lane == 63)
        scratch[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < waves; ++w) {
        const uint32_t v = scratch[w];
        if (w < wave)
            before += v;
        all += v;
    }
    *total = all;
    return before + incl - x;
}

} // namespace dev
} // namespace mcmf
