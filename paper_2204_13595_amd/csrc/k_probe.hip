// Measured ceilings of the GPU beside the published peaks that the roofline
// figures use: the rate of full-rate 32-bit integer VALU operations
// (independent 24-bit multiply-add chains in every lane, enough wavefronts to
// fill every SIMD) and the device-memory bandwidth of a streaming 16-byte copy.
#include "irbe_device.hpp"
#include "irbe_internal.hpp"

namespace irbe {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 8;   // independent chains per lane
constexpr int kProbeUnroll = 16;  // multiply-adds per chain per loop iteration

__global__ __launch_bounds__(kProbeBlock) void k_valu_probe(int iters, uint32_t seed, uint32_t* __restrict__ out)
{
    uint32_t a[kProbeChains];
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) a[k] = seed ^ (threadIdx.x * kProbeChains + k) ^ (blockIdx.x << 12);
    const uint32_t m = 0x9e37u ^ (seed & 1u), c = 0x7f4a7c15u;
    for (int it = 0; it < iters; ++it) {
        // one instruction per step, written as such: the compiler would otherwise
        // fold the affine chain into fewer (slower) full multiplies
#pragma unroll
        for (int u = 0; u < kProbeUnroll; ++u)
#pragma unroll
            for (int k = 0; k < kProbeChains; ++k) asm("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(a[k]) : "v"(m), "v"(c));
    }
    uint32_t x = 0;
#pragma unroll
    for (int k = 0; k < kProbeChains; ++k) x ^= a[k];
    out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = x;
}

// Four 16-byte loads in flight per thread, then their stores.
__global__ __launch_bounds__(kProbeBlock) void k_copy_probe(int64_t n, const uint4* __restrict__ src,
                                                           uint4* __restrict__ dst)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeBlock;
    int64_t i = (int64_t)blockIdx.x * kProbeBlock + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        const uint4 v0 = src[i], v1 = src[i + stride], v2 = src[i + 2 * stride], v3 = src[i + 3 * stride];
        dst[i] = v0;
        dst[i + stride] = v1;
        dst[i + 2 * stride] = v2;
        dst[i + 3 * stride] = v3;
    }
    for (; i < n; i += stride) dst[i] = src[i];
}

}  // namespace irbe

using namespace irbe;

namespace {

// Milliseconds of one launch of f on stream s (after one untimed launch).
template <typename F>
hipError_t time_launch(hipStream_t s, F f, float* ms)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) {
        f();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    if (e == hipSuccess) {
        f();
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return e;
}

}  // namespace

extern "C" irbe_status irbe_probe_rates(void* hip_stream, double* valu_lane_ops_per_s, double* copy_bytes_per_s)
{
    const hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                 hipSuccess)
        return IRBE_EHIP;
    if (valu_lane_ops_per_s) {
        // 32 wavefronts per CU, each lane 8 chains x 16 x iters multiply-adds
        const int blocks = cus * 8, iters = 2048;
        uint32_t* out = nullptr;
        if (hipMalloc(&out, (size_t)blocks * kProbeBlock * sizeof(uint32_t)) != hipSuccess) return IRBE_ENOMEM;
        float ms = 0.0f;
        const hipError_t e = time_launch(
            s, [&] { k_valu_probe<<<blocks, kProbeBlock, 0, s>>>(iters, 2204u, out); }, &ms);
        (void)hipFree(out);
        if (e != hipSuccess || !(ms > 0.0f)) return IRBE_EHIP;
        const double ops = (double)blocks * kProbeBlock * iters * kProbeUnroll * kProbeChains;
        *valu_lane_ops_per_s = ops / (ms * 1e-3);
    }
    if (copy_bytes_per_s) {
        const int64_t n = ((int64_t)1 << 30) / 16;  // 1 GiB
        uint4 *a = nullptr, *b = nullptr;
        if (hipMalloc(&a, (size_t)n * 16) != hipSuccess) return IRBE_ENOMEM;
        if (hipMalloc(&b, (size_t)n * 16) != hipSuccess) {
            (void)hipFree(a);
            return IRBE_ENOMEM;
        }
        hipError_t e = hipMemsetAsync(a, 0, (size_t)n * 16, s);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = time_launch(s, [&] { k_copy_probe<<<cus * 32, kProbeBlock, 0, s>>>(n, a, b); }, &ms);
        (void)hipFree(a);
        (void)hipFree(b);
        if (e != hipSuccess || !(ms > 0.0f)) return IRBE_EHIP;
        *copy_bytes_per_s = 2.0 * (double)n * 16.0 / (ms * 1e-3);  // bytes read + written
    }
    return IRBE_OK;
}
