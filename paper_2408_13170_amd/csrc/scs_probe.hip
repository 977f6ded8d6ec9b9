// Peak microbenchmark of the device: the ceilings the generate-and-reduce
// kernels are measured against, taken on the chip itself beside the
// published figures.  Four probes, each a grid of many waves per SIMD:
//   FP64 FMA      eight independent dependent chains per lane
//   FP32 FMA      the same in single precision (non-packed instructions)
//   FP32 sin      eight chains of the hardware sine (revolutions)
//   HBM copy      a streaming copy of 2 x 512 MiB (read plus write bytes)
// The chains end in a store guarded by a value the host never passes, so
// the compiler keeps them and nothing is written.
#include "scs.h"

#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr int kChains = 8;
constexpr int kIters = 1024;  // per lane and chain

__global__ __launch_bounds__(256) void k_fma64(double seed, double* sink, int never)
{
    double x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + threadIdx.x * 1e-9 + c;
    const double m = 0.999999, a = 1e-7;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fma(x[c], m, a);
    }
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (never == 0x5ca1ab1e) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_fma32(float seed, float* sink, int never)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + threadIdx.x * 1e-6f + c;
    const float m = 0.9999f, a = 1e-4f;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_fmaf(x[c], m, a);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (never == 0x5ca1ab1e) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_sin32(float seed, float* sink, int never)
{
    float x[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) x[c] = seed + threadIdx.x * 1e-6f + 0.01f * c;
    for (int i = 0; i < kIters; ++i) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) x[c] = __builtin_amdgcn_sinf(x[c]);
    }
    float s = 0.f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += x[c];
    if (never == 0x5ca1ab1e) sink[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

// the library's thread-local error record (scs_host.hip)
int scs_record_error(int code, const char* msg);

// out: [0] FP64 TFLOP/s, [1] FP32 TFLOP/s, [2] FP32 sines per second (1e12),
// [3] HBM copy TB/s (bytes read + written), [4] the device's clock as HIP
// reports it (GHz).
extern "C" int scs_peak_probe(int32_t device, double* out)
{
    if (!out) return scs_record_error(SCS_EINVAL, "out is NULL");
    if (hipSetDevice(device) != hipSuccess) return scs_record_error(SCS_EDEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return scs_record_error(SCS_EDEVICE, "hipGetDeviceProperties failed");
    const int n_cu = prop.multiProcessorCount;
    const int blocks = n_cu * 32;  // 8 waves per SIMD
    const int threads = 256;
    const int64_t bytes = (int64_t)512 << 20;
    const int64_t n4 = bytes / 16;
    float4 *src = nullptr, *dst = nullptr;
    double* sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipStream_t s = nullptr;
    int rc = SCS_OK;
    auto bad = [&](const char* what) {
        rc = scs_record_error(SCS_EDEVICE, what);
        return rc;
    };
    if (hipMalloc((void**)&src, bytes) != hipSuccess || hipMalloc((void**)&dst, bytes) != hipSuccess ||
        hipMalloc((void**)&sink, sizeof(double) * blocks * threads) != hipSuccess)
        rc = scs_record_error(SCS_ENOMEM, "peak probe: device allocation failed");
    if (!rc && (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess ||
                hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        bad("peak probe: stream or event creation failed");
    if (!rc && hipMemsetAsync(src, 0, bytes, s) != hipSuccess) bad("peak probe: memset failed");
    // time(kernel) in ms: one warm-up launch, then the mean of three
    auto timed = [&](auto launch) -> double {
        if (rc) return 0.0;
        launch();
        if (hipEventRecord(e0, s) != hipSuccess) return bad("peak probe: event record failed"), 0.0;
        for (int r = 0; r < 3; ++r) launch();
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return bad("peak probe: event wait failed"), 0.0;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return bad("peak probe: event timing failed"), 0.0;
        return ms / 3.0;
    };
    const double lanes = (double)blocks * threads;
    const double ops = lanes * kChains * kIters;  // FMA or sine per probe launch
    const double t64 = timed([&] { hipLaunchKernelGGL(k_fma64, dim3(blocks), dim3(threads), 0, s, 1.0, sink, 0); });
    const double t32 = timed([&] {
        hipLaunchKernelGGL(k_fma32, dim3(blocks), dim3(threads), 0, s, 1.0f, (float*)sink, 0);
    });
    const double tsin = timed([&] {
        hipLaunchKernelGGL(k_sin32, dim3(blocks), dim3(threads), 0, s, 0.1f, (float*)sink, 0);
    });
    const double tcp = timed([&] { hipLaunchKernelGGL(k_copy, dim3(n_cu * 16), dim3(256), 0, s, src, dst, n4); });
    if (!rc && hipGetLastError() != hipSuccess) bad("peak probe: kernel launch failed");
    if (!rc) {
        out[0] = 2.0 * ops / (t64 * 1e-3) / 1e12;
        out[1] = 2.0 * ops / (t32 * 1e-3) / 1e12;
        out[2] = ops / (tsin * 1e-3) / 1e12;
        out[3] = 2.0 * (double)bytes / (tcp * 1e-3) / 1e12;
        out[4] = prop.clockRate / 1e6;
    }
    if (s) hipStreamSynchronize(s);
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    if (s) hipStreamDestroy(s);
    hipFree(src);
    hipFree(dst);
    hipFree(sink);
    return rc;
}
