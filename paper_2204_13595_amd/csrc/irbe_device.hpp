// Device-side building blocks: counter-based random numbers, bounded integers,
// wavefront/block reductions and precision traits.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace irbe {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplications with the Weyl key schedule.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Words4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                           uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c1 ^ k0;
        const uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return {c0, c1, c2, c3};
}

// Word stream: block b = Philox({c0, b, step lo, (step hi << 1) | tag}, seed).
struct WordStream {
    uint32_t k0, k1, c0, c2, c3, block;
    Words4 buf;
    int pos;

    __device__ __forceinline__ WordStream(uint64_t seed, uint64_t step, uint32_t id, uint32_t tag)
        : k0((uint32_t)seed), k1((uint32_t)(seed >> 32)), c0(id), c2((uint32_t)step),
          c3(((uint32_t)(step >> 32) << 1) | (tag & 1u)), block(0), buf{0, 0, 0, 0}, pos(4)
    {
    }

    __device__ __forceinline__ uint32_t next()
    {
        if (pos == 4) {
            buf = philox10(c0, block, c2, c3, k0, k1);
            ++block;
            pos = 0;
        }
        const uint32_t v = pos == 0 ? buf.x : pos == 1 ? buf.y : pos == 2 ? buf.z : buf.w;
        ++pos;
        return v;
    }

    // Uniform in [0, n), n >= 1 (Lemire 2019, multiply-shift with rejection).
    __device__ __forceinline__ uint32_t below(uint32_t n)
    {
        uint64_t m = (uint64_t)next() * (uint64_t)n;
        uint32_t l = (uint32_t)m;
        if (l < n) {
            const uint32_t thr = (0u - n) % n;
            while (l < thr) {
                m = (uint64_t)next() * (uint64_t)n;
                l = (uint32_t)m;
            }
        }
        return (uint32_t)(m >> 32);
    }
};

// Workgroups are dispatched round-robin over the XCDs (8 on MI355X), each with
// its own L2. Mapping hardware block b to logical block xcd_block(b) gives every
// XCD one contiguous range of logical blocks, i.e. one compact region of the
// cell-sorted atoms, so the neighbour data an XCD reads stays in its own L2. A
// bijection of [0, nb) for any nb.
constexpr int kNumXcd = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nb)
{
    const int64_t x = b % kNumXcd, i = b / kNumXcd;
    const int64_t q = nb / kNumXcd, r = nb % kNumXcd;
    return x * q + (x < r ? x : r) + i;
}

constexpr uint32_t kTagShell = 0u;
constexpr uint32_t kTagKspace = 1u;

// Value of v in lane t (t uniform across the wavefront): v_readlane into a scalar.
__device__ __forceinline__ int bcast(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ __forceinline__ uint32_t bcast(uint32_t v, int t) { return (uint32_t)__builtin_amdgcn_readlane((int)v, t); }
__device__ __forceinline__ float bcast(float v, int t)
{
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), t));
}
__device__ __forceinline__ double bcast(double v, int t)
{
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), t);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), t);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// Reductions (fixed order: deterministic for a fixed launch shape).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_sum(T v)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums NV values per thread over a block of BLOCK threads; thread v < NV of the
// block receives total v in the return value (others: 0). lds: NV * (BLOCK/64).
template <int NV, int BLOCK>
__device__ __forceinline__ double block_sum_vec(double* vals, double* lds, int v_out_idx, double& out)
{
    constexpr int NW = BLOCK / 64;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double s = wave_sum(vals[v]);
        if (lane == 0) lds[v * NW + wave] = s;
    }
    __syncthreads();
    out = 0.0;
    if (v_out_idx < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < NW; ++w) t += lds[v_out_idx * NW + w];
        out = t;
    }
    __syncthreads();
    return out;
}

// ---------------------------------------------------------------------------
// Precision traits.
// ---------------------------------------------------------------------------
template <typename real>
struct Math;

template <>
struct Math<float> {
    static __device__ __forceinline__ float max_() { return 3.402823466e38f; }
    static __device__ __forceinline__ float erfc_(float x) { return erfcf(x); }
    // erfc(x) for x >= 0 given ex = exp(-x^2): the Chebyshev-fitted form of
    // Numerical Recipes (Press et al., Sec. 6.2, "erfcc"), fractional error
    // below 1.2e-7: erfc(x) = t exp(-x^2 + P(t)), t = 1/(1 + x/2).
    static __device__ __forceinline__ float erfc_ex(float x, float ex)
    {
        const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
        float p = 0.17087277f;
        p = fmaf(p, t, -0.82215223f);
        p = fmaf(p, t, 1.48851587f);
        p = fmaf(p, t, -1.13520398f);
        p = fmaf(p, t, 0.27886807f);
        p = fmaf(p, t, -0.18628806f);
        p = fmaf(p, t, 0.09678418f);
        p = fmaf(p, t, 0.37409196f);
        p = fmaf(p, t, 1.00002368f);
        p = fmaf(p, t, -1.26551223f);
        return t * ex * __expf(p);
    }
    static __device__ __forceinline__ float erf_(float x) { return erff(x); }
    static __device__ __forceinline__ float exp_(float x) { return __expf(x); }
    // the hardware reciprocal square root: the arguments are squared pair
    // separations, far from the denormal range that rsqrtf rescales for
    static __device__ __forceinline__ float rsqrt_(float x) { return __builtin_amdgcn_rsqf(x); }
    static __device__ __forceinline__ float sqrt_(float x) { return sqrtf(x); }
    // sin and cos of 2 pi x for a phase x in revolutions, |x| <= 1/2.
    static __device__ __forceinline__ void sincos_rev(float x, float* s, float* c)
    {
        *s = __builtin_amdgcn_sinf(x);
        *c = __builtin_amdgcn_cosf(x);
    }
};

template <>
struct Math<double> {
    static __device__ __forceinline__ double max_() { return 1.7976931348623157e308; }
    static __device__ __forceinline__ double erfc_(double x) { return erfc(x); }
    static __device__ __forceinline__ double erfc_ex(double x, double) { return erfc(x); }
    static __device__ __forceinline__ double erf_(double x) { return erf(x); }
    static __device__ __forceinline__ double exp_(double x) { return exp(x); }
    static __device__ __forceinline__ double rsqrt_(double x) { return rsqrt(x); }
    static __device__ __forceinline__ double sqrt_(double x) { return sqrt(x); }
    static __device__ __forceinline__ void sincos_rev(double x, double* s, double* c) { sincospi(2.0 * x, s, c); }
};

// Exact k.r phase: (m . s) mod 2^32, returned in revolutions in [-1/2, 1/2).
template <typename real>
__device__ __forceinline__ real phase_rev(int mx, int my, int mz, uint32_t sx, uint32_t sy, uint32_t sz)
{
    const uint32_t ph = (uint32_t)mx * sx + (uint32_t)my * sy + (uint32_t)mz * sz;
    return (real)(int32_t)ph * (real)2.3283064365386963e-10;  // 2^-32
}

}  // namespace irbe
