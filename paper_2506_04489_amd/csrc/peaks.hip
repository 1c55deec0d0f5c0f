// peaks.hip - the two ceilings the kernels are measured against, taken on
// the device at hand: a streaming copy (HBM bandwidth) and back-to-back
// FP64 MFMA instructions (matrix-core rate).
#include <algorithm>
#include <vector>

#include "host_common.hpp"

namespace psp {

typedef double v4d_peak __attribute__((ext_vector_type(4)));

// dst[i] = src[i] over `count` 16-byte elements: each thread loads four
// elements a block-width apart before storing them, grid-stride
__global__ void __launch_bounds__(256) k_peak_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   size_t count) {
    const size_t step = (size_t)blockDim.x, stride = (size_t)gridDim.x * step * 4;
    for (size_t base = (size_t)blockIdx.x * step * 4 + threadIdx.x; base < count; base += stride) {
        double2 v[4];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k * step < count) v[k] = src[base + k * step];
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (base + k * step < count) dst[base + k * step] = v[k];
    }
}

// every wave: `iters` rounds of PEAK_ACC independent 16x16x4 FP64 MFMAs
// (2048 flops each); the result is stored only if it matches an impossible
// value, so the chains stay live without memory traffic
constexpr int PEAK_ACC = 8;
__global__ void __launch_bounds__(256) k_peak_mfma(double *out, int iters, double seed) {
    v4d_peak acc[PEAK_ACC];
    for (int k = 0; k < PEAK_ACC; ++k) acc[k] = v4d_peak{0.0, 0.0, 0.0, 0.0};
    const double a = seed * (threadIdx.x + 1), b = 1.0 / (blockIdx.x + 2.0);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < PEAK_ACC; ++k) acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[k], 0, 0, 0);
    }
    double s = 0.0;
    for (int k = 0; k < PEAK_ACC; ++k) s += acc[k][k & 3];
    if (s == -1.2345e300) out[blockIdx.x] = s;
}

}  // namespace psp

using namespace psp;

extern "C" psp_status psp_device_peaks(void *buf_a, void *buf_b, size_t bytes, void *stream, double *copy_gbps,
                                       double *fp64_mfma_tflops) {
    return guarded([&]() -> psp_status {
        if (!buf_a || !buf_b || !copy_gbps || !fp64_mfma_tflops) return fail(PSP_EINVAL, "NULL argument");
        if (bytes < (1u << 20) || (bytes & 15)) return fail(PSP_EINVAL, "bytes must be >= 1 MiB and a multiple of 16");
        hipStream_t st = (hipStream_t)stream;
        int dev = -1, cus = 0;
        hipError_t he = hipGetDevice(&dev);
        if (he == hipSuccess) he = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (he != hipSuccess) return hip_fail(he, "device query");
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if ((he = hipEventCreate(&e0)) != hipSuccess) return hip_fail(he, "hipEventCreate");
        if ((he = hipEventCreate(&e1)) != hipSuccess) {
            (void)hipEventDestroy(e0);
            return hip_fail(he, "hipEventCreate");
        }
        psp_status out = PSP_OK;
        auto timed = [&](auto launch, int reps, float *best) -> hipError_t {
            hipError_t e = hipSuccess;
            *best = 1e30f;
            for (int r = 0; r < reps + 1 && e == hipSuccess; ++r) {   // the first run warms up
                if ((e = hipEventRecord(e0, st)) != hipSuccess) break;
                launch();
                if ((e = hipGetLastError()) != hipSuccess || (e = hipEventRecord(e1, st)) != hipSuccess ||
                    (e = hipEventSynchronize(e1)) != hipSuccess)
                    break;
                float ms = 0;
                if ((e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess) break;
                if (r > 0) *best = std::min(*best, ms);
            }
            return e;
        };
        const size_t count = bytes / 16;
        float ms = 0;
        hipError_t e = timed(
            [&] {
                hipLaunchKernelGGL(k_peak_copy, dim3(cus * 16), dim3(256), 0, st, (const double2 *)buf_a, (double2 *)buf_b,
                                   count);
            },
            5, &ms);
        if (e != hipSuccess) out = hip_fail(e, "copy peak");
        else *copy_gbps = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
        if (out == PSP_OK) {
            const int iters = 2048, blocks = cus * 8;    // 4 waves per block
            e = timed([&] { hipLaunchKernelGGL(k_peak_mfma, dim3(blocks), dim3(256), 0, st, (double *)buf_b, iters, 1e-3); },
                      5, &ms);
            if (e != hipSuccess) out = hip_fail(e, "MFMA peak");
            else *fp64_mfma_tflops = (double)blocks * 4 * iters * PEAK_ACC * 2048.0 / (ms * 1e-3) / 1e12;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return out;
    });
}
