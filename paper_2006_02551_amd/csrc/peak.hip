// Measurement helpers for the roofline's measured peaks: the sustained rate of the matrix-core
// instruction the stage kernel uses (FP64: V_MFMA_F64_4X4X4_4B_F64, FP32: V_MFMA_F32_16X16X4_F32), and the
// device-memory bandwidth of a plain copy.
//
// Every wavefront runs independent accumulator chains of `iters` MFMAs each, so the matrix pipe of a SIMD
// always has independent work; the grid puts several workgroups on every compute unit.  The accumulators
// are written out at the end so that nothing is dead code.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/wdg.h"

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kChains = 8;
constexpr int kThreads = 256;  // four wavefronts per workgroup

template <typename real>
struct PeakMma;
template <>
struct PeakMma<double> {  // four four-block 4x4x4 products = one 16x16x4 step, as the stage kernel issues them
    using v4 = v4d;
    static __device__ __forceinline__ v4 run(double a, double b, v4 c) {
#pragma unroll
        for (int v = 0; v < 4; ++v) c[v] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c[v], 0, 0, 0);
        return c;
    }
};
template <>
struct PeakMma<float> {
    using v4 = v4f;
    static __device__ __forceinline__ v4 run(float a, float b, v4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <typename real>
__global__ __launch_bounds__(kThreads) void mfma_peak_kernel(real* out, int iters) {
    using v4 = typename PeakMma<real>::v4;
    const int lane = static_cast<int>(threadIdx.x) & 63;
    // operands near 1: every MFMA adds about 4 to each accumulator, finite for any practical count
    const real a = real(1) + real(lane) * real(1e-7), b = real(1) - real(lane) * real(1e-7);
    v4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = v4{real(c), 0, 0, 0};
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = PeakMma<real>::run(a, b, acc[c]);
    }
    real s = 0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[static_cast<size_t>(blockIdx.x) * kThreads + threadIdx.x] = s;
}

}  // namespace

extern "C" int32_t wdg_measure_mfma_peak(int32_t precision, int32_t iters, void* hip_stream, double* tflops) {
    if (!tflops || iters <= 0 || (precision != WDG_FP64 && precision != WDG_FP32)) return WDG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return WDG_EHIP;
    const int blocks = 8 * cus;
    const size_t rb = precision == WDG_FP64 ? 8 : 4;
    void* out = nullptr;
    if (hipMalloc(&out, static_cast<size_t>(blocks) * kThreads * rb) != hipSuccess) return WDG_ENOMEM;
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 0.0f;
    int32_t rc = WDG_OK;
    for (int rep = 0; rep < 4 && rc == WDG_OK; ++rep) {  // the first launch also loads the code object
        (void)hipEventRecord(e0, s);
        if (precision == WDG_FP64)
            hipLaunchKernelGGL(mfma_peak_kernel<double>, dim3(blocks), dim3(kThreads), 0, s, static_cast<double*>(out), iters);
        else
            hipLaunchKernelGGL(mfma_peak_kernel<float>, dim3(blocks), dim3(kThreads), 0, s, static_cast<float*>(out), iters);
        (void)hipEventRecord(e1, s);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = WDG_EHIP;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(out);
    if (rc != WDG_OK) return rc;
    // one 16x16x4 step per wavefront is 16 * 16 * 4 multiply-adds
    const double flops = 2.0 * 16 * 16 * 4 * static_cast<double>(kChains) * iters * (static_cast<double>(blocks) * kThreads / 64);
    *tflops = flops / (static_cast<double>(best) * 1e-3) / 1e12;
    return WDG_OK;
}

namespace {

constexpr int kCopyUnroll = 4;

__global__ __launch_bounds__(256) void copy_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
    const size_t base = static_cast<size_t>(blockIdx.x) * (256 * kCopyUnroll) + threadIdx.x;
    uint4 v[kCopyUnroll];
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + static_cast<size_t>(u) * 256;
        if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
        const size_t i = base + static_cast<size_t>(u) * 256;
        if (i < n) dst[i] = v[u];
    }
}

}  // namespace

extern "C" int32_t wdg_measure_copy_bandwidth(int64_t bytes, void* hip_stream, double* gbs) {
    if (!gbs || bytes < (1 << 20) || bytes % 16 != 0) return WDG_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, static_cast<size_t>(bytes)) != hipSuccess) return WDG_ENOMEM;
    if (hipMalloc(&dst, static_cast<size_t>(bytes)) != hipSuccess) {
        (void)hipFree(src);
        return WDG_ENOMEM;
    }
    int32_t rc = hipMemsetAsync(src, 0, static_cast<size_t>(bytes), s) == hipSuccess ? WDG_OK : WDG_EHIP;
    const size_t n = static_cast<size_t>(bytes) / 16;
    const unsigned blocks = static_cast<unsigned>((n + 256 * kCopyUnroll - 1) / (256 * kCopyUnroll));
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    float best = 0.0f;
    for (int rep = 0; rep < 6 && rc == WDG_OK; ++rep) {  // the first launch is untimed
        (void)hipEventRecord(e0, s);
        hipLaunchKernelGGL(copy_kernel, dim3(blocks), dim3(256), 0, s, static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
        (void)hipEventRecord(e1, s);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
            rc = WDG_EHIP;
            break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (rep > 0 && (best == 0.0f || ms < best)) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(src);
    (void)hipFree(dst);
    if (rc != WDG_OK) return rc;
    *gbs = 2.0 * static_cast<double>(bytes) / (static_cast<double>(best) * 1e-3) / 1e9;
    return WDG_OK;
}
