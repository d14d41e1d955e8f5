// pn_probe.hip -- sustained vector FMA rate of the device, the measured
// counterpart of the datasheet peaks the roofline figures are quoted
// against.  Eight independent multiply-add chains per lane (no dependence
// between consecutive instructions of a chain), FP32 without packed
// instructions and FP64, over a grid of the requested waves per SIMD.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pn.h"

namespace pn {
int device_ready();   // pn_lib.hip: PN_OK when a gfx950 device is current

namespace {

constexpr int kProbeBlock = 256;   // 4 waves: one per SIMD of a CU
constexpr int kUnroll = 16;        // chain steps per loop iteration

template <class T>
__global__ __launch_bounds__(kProbeBlock) void fma_chains(T* __restrict__ out, int iters, T a, T b) {
    T x0 = (T)threadIdx.x, x1 = x0 + (T)1, x2 = x0 + (T)2, x3 = x0 + (T)3;
    T x4 = x0 + (T)4, x5 = x0 + (T)5, x6 = x0 + (T)6, x7 = x0 + (T)7;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < kUnroll; ++k) {
            x0 = x0 * a + b; x1 = x1 * a + b; x2 = x2 * a + b; x3 = x3 * a + b;
            x4 = x4 * a + b; x5 = x5 * a + b; x6 = x6 * a + b; x7 = x7 * a + b;
        }
    }
    // keeps the chains live; one element per thread of the grid
    out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

// The FP64 chains on the first `active` lanes of every wave only (the rest
// skip the loop under the execution mask): a known number of lane FLOPs for
// calibrating instruction and FLOP counters on partly active waves.
__global__ __launch_bounds__(kProbeBlock) void fma_chains_lanes(double* __restrict__ out, int iters, double a,
                                                                double b, int active) {
    double x0 = (double)threadIdx.x, x1 = x0 + 1.0, x2 = x0 + 2.0, x3 = x0 + 3.0;
    double x4 = x0 + 4.0, x5 = x0 + 5.0, x6 = x0 + 6.0, x7 = x0 + 7.0;
    if ((int)(threadIdx.x % 64) < active) {
        for (int i = 0; i < iters; ++i) {
#pragma unroll
            for (int k = 0; k < kUnroll; ++k) {
                x0 = x0 * a + b; x1 = x1 * a + b; x2 = x2 * a + b; x3 = x3 * a + b;
                x4 = x4 * a + b; x5 = x5 * a + b; x6 = x6 * a + b; x7 = x7 * a + b;
            }
        }
    }
    out[(int64_t)blockIdx.x * kProbeBlock + threadIdx.x] = ((x0 + x1) + (x2 + x3)) + ((x4 + x5) + (x6 + x7));
}

template <class T>
int time_chains(int blocks, int iters, hipStream_t s, double* tflops) {
    T* out = nullptr;
    if (hipMalloc(&out, sizeof(T) * (size_t)blocks * kProbeBlock) != hipSuccess) return PN_ENOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PN_OK;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = PN_EHIP;
    float ms = 0.0f;
    if (rc == PN_OK) {
        // one warm-up launch, then the timed one
        hipLaunchKernelGGL(fma_chains<T>, dim3(blocks), dim3(kProbeBlock), 0, s, out, iters, (T)0.999, (T)0.001);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e0, s) != hipSuccess) rc = PN_EHIP;
    }
    if (rc == PN_OK) {
        hipLaunchKernelGGL(fma_chains<T>, dim3(blocks), dim3(kProbeBlock), 0, s, out, iters, (T)0.999, (T)0.001);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
            rc = PN_EHIP;
    }
    if (rc == PN_OK) {
        const double flop = 2.0 * 8.0 * kUnroll * (double)iters * (double)blocks * kProbeBlock;
        *tflops = ms > 0.0f ? flop / ((double)ms * 1e-3) / 1e12 : 0.0;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}

}  // namespace
}  // namespace pn

extern "C" int pn_fma_rate(int32_t waves_per_simd, int32_t iters, double* fp32_tflops, double* fp64_tflops,
                           void* stream) {
    if (waves_per_simd < 1 || waves_per_simd > 8 || iters < 1 || iters > (1 << 20) || !fp32_tflops ||
        !fp64_tflops)
        return PN_EINVAL;
    const int ready = pn::device_ready();
    if (ready != PN_OK) return ready;
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return PN_ENODEV;
    const int blocks = cus * waves_per_simd;
    hipStream_t s = (hipStream_t)stream;
    int rc = pn::time_chains<float>(blocks, iters, s, fp32_tflops);
    if (rc == PN_OK) rc = pn::time_chains<double>(blocks, iters, s, fp64_tflops);
    return rc;
}

extern "C" int pn_fma_lanes(int32_t active_lanes, int32_t iters, double* lane_flop, double* ms, void* stream) {
    if (active_lanes < 0 || active_lanes > 64 || iters < 1 || iters > (1 << 20) || !lane_flop || !ms)
        return PN_EINVAL;
    const int ready = pn::device_ready();
    if (ready != PN_OK) return ready;
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
        return PN_ENODEV;
    const int blocks = cus;            // one wave per SIMD
    hipStream_t s = (hipStream_t)stream;
    double* out = nullptr;
    if (hipMalloc(&out, sizeof(double) * (size_t)blocks * pn::kProbeBlock) != hipSuccess) return PN_ENOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = PN_OK;
    float t = 0.0f;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = PN_EHIP;
    if (rc == PN_OK && hipEventRecord(e0, s) != hipSuccess) rc = PN_EHIP;
    if (rc == PN_OK) {
        hipLaunchKernelGGL(pn::fma_chains_lanes, dim3(blocks), dim3(pn::kProbeBlock), 0, s, out, iters, 0.999, 0.001,
                           (int)active_lanes);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, s) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&t, e0, e1) != hipSuccess)
            rc = PN_EHIP;
    }
    if (rc == PN_OK) {
        *lane_flop = 2.0 * 8.0 * pn::kUnroll * (double)iters * (double)blocks * (pn::kProbeBlock / 64) * active_lanes;
        *ms = t;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
