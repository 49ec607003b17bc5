// Device helpers shared by the library's kernels (wave64 reductions,
// deterministic block partials).
#pragma once

#include <hip/hip_runtime.h>

namespace dect {

constexpr int kWave = 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}
// Minimum / maximum of an int over the wavefront, returned in every lane
// (wave-uniform).  Within each row of 16 lanes by DPP: the two quad
// butterflies (quad_perm [1,0,3,2] and [2,3,0,1]), then the half-row and row
// mirrors, after which every lane of a row holds the row's result; then the
// four rows through readlane.  All 64 lanes must be active.
template <typename Op>
__device__ __forceinline__ int wave_reduce_i32(int v, Op op) {
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false));    // quad_perm [1,0,3,2]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false));    // quad_perm [2,3,0,1]
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false));   // row_half_mirror
    v = op(v, __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false));   // row_mirror
    const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
    const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
    return op(op(a, b), op(c, d));
}
__device__ __forceinline__ int wave_min(int v) {
    return wave_reduce_i32(v, [](int x, int y) { return min(x, y); });
}
__device__ __forceinline__ int wave_max(int v) {
    return wave_reduce_i32(v, [](int x, int y) { return max(x, y); });
}

// Sum of `v` over a 1-D block of NT threads, fixed order; result valid in
// thread 0.  `sh` holds NT/64 doubles of LDS.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
    v = wave_sum(v);
    const int w = threadIdx.x / kWave;
    if ((threadIdx.x % kWave) == 0) sh[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int i = 0; i < NT / kWave; ++i) r += sh[i];
    }
    __syncthreads();
    return r;
}

// Sums of N values per thread over a 1-D block of NT threads in one LDS
// round, fixed order; results broadcast to every thread.  `sh` holds
// N * NT/64 doubles of LDS.
template <int NT, int N>
__device__ __forceinline__ void block_sum_n(double (&v)[N], double* sh) {
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int c = 0; c < N; ++c) {
        const double t = wave_sum(v[c]);
        if ((threadIdx.x % kWave) == 0) sh[c * (NT / kWave) + w] = t;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < N; ++c) {
        double r = 0.0;
#pragma unroll
        for (int i = 0; i < NT / kWave; ++i) r += sh[c * (NT / kWave) + i];
        v[c] = r;
    }
    __syncthreads();
}

// Deterministic sum of n doubles at stride `stride` (fixed tree order), done
// by all threads of a block of NT threads; result valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum_array(const double* a, int n, int stride, double* sh) {
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) v += a[(size_t)i * stride];
    return block_sum<NT>(v, sh);
}

// BF16 storage: two values in one 32-bit word, x in the low half.  Rounding
// to nearest, ties to even (finite inputs); widening is exact.
__device__ __forceinline__ unsigned bf16_bits(float x) {
    const unsigned u = __float_as_uint(x);
    return (u + 0x7fffu + ((u >> 16) & 1u)) >> 16;
}
__device__ __forceinline__ unsigned bf16x2_pack(float x, float y) {
    return bf16_bits(x) | (bf16_bits(y) << 16);
}
__device__ __forceinline__ float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }
__device__ __forceinline__ float2 bf16x2_unpack(unsigned w) { return make_float2(bf16_lo(w), bf16_hi(w)); }
__device__ __forceinline__ float bf16_round(float x) { return __uint_as_float(bf16_bits(x) << 16); }

// Stochastic rounding to BF16 for values that accumulate small updates (the
// residual sinograms, the state images): adding 16 uniform random bits below
// the kept ones before truncating rounds the magnitude up with probability
// equal to the dropped fraction, so the stored value is unbiased and an update
// below half a BF16 ulp survives in expectation instead of being rounded away.
// Non-finite inputs round to nearest.  The bits come from the finaliser of
// MurmurHash3 (Appleby) over an element index and a per-slice seed, so the
// rounding is deterministic.
__device__ __forceinline__ unsigned fmix32(unsigned h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
__device__ __forceinline__ unsigned seed_of(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return fmix32((unsigned)b ^ fmix32((unsigned)(b >> 32)));
}
__device__ __forceinline__ unsigned bf16_bits_sr(float x, unsigned r16) {
    const unsigned u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return bf16_bits(x);
    return (u + (r16 & 0xffffu)) >> 16;
}
// x takes the low 16 random bits, y the high 16
__device__ __forceinline__ unsigned bf16x2_pack_sr(float x, float y, unsigned r) {
    return bf16_bits_sr(x, r) | (bf16_bits_sr(y, r >> 16) << 16);
}
__device__ __forceinline__ float bf16_round_sr(float x, unsigned r16) {
    return __uint_as_float(bf16_bits_sr(x, r16) << 16);
}

__device__ __forceinline__ int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

}  // namespace dect
