// Device ceilings for the roofline: a sustained FP64 MFMA rate and a copy
// bandwidth, measured on the device the library runs on (the published
// MI355X figures are 78.6 TFLOP/s FP64 matrix and 8 TB/s HBM).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "selinv.h"

namespace {
typedef double pd4 __attribute__((ext_vector_type(4)));
typedef double pd2 __attribute__((ext_vector_type(2)));

constexpr int kProbeThreads = 256;
constexpr int kChains = 8;  // independent accumulators per wave: the MFMA pipe never waits on a result

// Every wave issues iters x kChains back-to-back v_mfma_f64_16x16x4f64 on
// independent accumulators (2 * 16 * 16 * 4 flops each); the sums are
// stored so nothing is dropped.
__global__ __launch_bounds__(kProbeThreads) void k_mfma_peak(double* __restrict__ out, int iters, double seed)
{
    const int lane = threadIdx.x & 63;
    double a = seed + 1e-3 * lane, b = seed - 1e-3 * lane;
    pd4 acc[kChains];
#pragma unroll
    for (int c = 0; c < kChains; ++c) acc[c] = pd4{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < kChains; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
        a += 1e-9;
    }
    __builtin_amdgcn_sched_barrier(0);
    asm volatile("s_nop 15\n\ts_nop 15\n\ts_nop 15\n\ts_nop 15" ::: "memory");
    __builtin_amdgcn_sched_barrier(0);
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
    out[blockIdx.x * (int64_t)kProbeThreads + threadIdx.x] = s;
}

// dst = src: each thread moves four 16-byte elements per iteration (all four
// loads issued before the stores), grid-stride; the tail element by element
__global__ __launch_bounds__(kProbeThreads) void k_copy(const pd2* __restrict__ src, pd2* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * kProbeThreads;
    const int64_t n4 = n / (4 * stride) * (4 * stride);
    for (int64_t i = blockIdx.x * (int64_t)kProbeThreads + threadIdx.x; i < n4; i += 4 * stride) {
        const pd2 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
        dst[i] = a;
        dst[i + stride] = b;
        dst[i + 2 * stride] = c;
        dst[i + 3 * stride] = d;
    }
    for (int64_t i = n4 + blockIdx.x * (int64_t)kProbeThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

thread_local std::string g_probe_err;
}  // namespace

extern "C" selinv_status selinv_measure_peaks(void* d_buf, size_t bytes, double* fp64_mfma_tflops, double* copy_gbs,
                                              hipStream_t s)
{
    const size_t kMin = (size_t)64 << 20;
    if (!d_buf || bytes < kMin || ((uintptr_t)d_buf & 255) != 0) return SELINV_EINVAL;
    hipDeviceProp_t prop;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (!e) e = hipGetDeviceProperties(&prop, dev);
    if (e) return SELINV_EHIP;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess) return SELINV_EHIP;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return SELINV_EHIP;
    }
    // MFMA: 8 work-groups (32 waves) per compute unit
    const int groups = prop.multiProcessorCount * 8, iters = 4000;
    const double flops = (double)groups * (kProbeThreads / 64) * iters * kChains * 2.0 * 16 * 16 * 4;
    double best_tf = 0.0, best_gbs = 0.0;
    for (int r = 0; r < 4 && !e; r++) {
        hipLaunchKernelGGL(k_mfma_peak, dim3(groups), dim3(kProbeThreads), 0, s, (double*)d_buf, iters, 1.0 + r);
        e = hipGetLastError();
        if (!e) e = hipEventRecord(e0, s);
        hipLaunchKernelGGL(k_mfma_peak, dim3(groups), dim3(kProbeThreads), 0, s, (double*)d_buf, iters, 2.0 + r);
        if (!e) e = hipGetLastError();
        if (!e) e = hipEventRecord(e1, s);
        if (!e) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (!e) e = hipEventElapsedTime(&ms, e0, e1);
        if (!e && ms > 0.f) best_tf = std::max(best_tf, flops / (ms * 1e-3) / 1e12);
    }
    // copy: first half of the buffer into the second half
    const int64_t n = (int64_t)(bytes / 2 / sizeof(pd2));
    const pd2* src = (const pd2*)d_buf;
    pd2* dst = (pd2*)d_buf + n;
    const int cgroups = prop.multiProcessorCount * 8;
    for (int r = 0; r < 5 && !e; r++) {
        e = hipEventRecord(e0, s);
        hipLaunchKernelGGL(k_copy, dim3(cgroups), dim3(kProbeThreads), 0, s, src, dst, n);
        if (!e) e = hipGetLastError();
        if (!e) e = hipEventRecord(e1, s);
        if (!e) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (!e) e = hipEventElapsedTime(&ms, e0, e1);
        if (!e && ms > 0.f && r > 0) best_gbs = std::max(best_gbs, 2.0 * n * sizeof(pd2) / (ms * 1e-3) / 1e9);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e) return SELINV_EHIP;
    if (fp64_mfma_tflops) *fp64_mfma_tflops = best_tf;
    if (copy_gbs) *copy_gbs = best_gbs;
    return SELINV_OK;
}
