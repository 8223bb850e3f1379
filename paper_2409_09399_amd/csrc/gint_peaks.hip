// Achievable peak rates of the units the grid-integration kernels use, measured
// on the current device: FP64 MFMA (v_mfma_f64_16x16x4f64), FP16 MFMA
// (v_mfma_f32_16x16x32_f16), FP32 and FP64 vector FMA.  Each kernel runs
// independent dependency chains per wave (enough to cover the instruction
// latency) on every SIMD of every CU; the result is flops / elapsed time of
// the launch.  These are the "measured" denominators beside the datasheet
// peaks when a kernel's roofline fraction is reported.
#include <hip/hip_runtime.h>

#include "gint_peaks.h"

typedef double d4p __attribute__((ext_vector_type(4)));
typedef float f4p __attribute__((ext_vector_type(4)));
typedef _Float16 h8p __attribute__((ext_vector_type(8)));

namespace {

constexpr int kIters = 2048;
constexpr int kChains = 4;

__global__ __launch_bounds__(256) void k_peak_mfma64(double seed, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    double a = seed + lane * 1e-3, b = seed - lane * 1e-3;
    d4p c[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) c[k] = (d4p){0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c[k], 0, 0, 0);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    if (s == 12345.678) out[blockIdx.x] = s;   // keeps the chains live; never true for the seeds used
}

__global__ __launch_bounds__(256) void k_peak_mfma16(float seed, double *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    h8p a, b;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        a[e] = (_Float16)(seed + 1e-3f * (lane + e));
        b[e] = (_Float16)(seed - 1e-3f * (lane + e));
    }
    f4p c[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) c[k] = (f4p){0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) c[k] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c[k], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kChains; ++k) s += c[k][0] + c[k][1] + c[k][2] + c[k][3];
    if (s == 12345.678f) out[blockIdx.x] = s;
}

__device__ inline float fma_t(float x, float m, float a) { return __builtin_fmaf(x, m, a); }
__device__ inline double fma_t(double x, double m, double a) { return __builtin_fma(x, m, a); }

template <class T>
__global__ __launch_bounds__(256) void k_peak_fma(T seed, double *__restrict__ out) {
    constexpr int kV = 8;   // independent chains per lane
    T x[kV];
    const T m = (T)0.999999, a = (T)1e-7;
#pragma unroll
    for (int k = 0; k < kV; ++k) x[k] = seed + (T)(threadIdx.x + k);
    for (int it = 0; it < kIters; ++it) {
#pragma unroll
        for (int k = 0; k < kV; ++k) x[k] = fma_t(x[k], m, a);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < kV; ++k) s += x[k];
    if (s == (T)12345.678) out[blockIdx.x] = (double)s;
}

int cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    return cus;
}

}  // namespace

extern "C" int gint_peaks_measure(double *tflops, void *stream) {
    if (!tflops) return -1;
    hipStream_t s = (hipStream_t)stream;
    const int cus = cu_count();
    if (cus <= 0) return -4;
    // 8 workgroups of 4 waves per CU: 8 waves per SIMD
    const int blocks = cus * 8;
    double *out = nullptr;
    if (hipMalloc(&out, sizeof(double) * blocks) != hipSuccess) return -3;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = 0;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) rc = -4;
    const double waves = (double)blocks * 4.0;
    // flops per wave: MFMA 16x16x4 f64 = 2048, 16x16x32 f16 = 16384 per instruction;
    // vector FMA = 2 x 64 lanes per instruction
    const double fl[4] = {waves * kIters * kChains * 2048.0, waves * kIters * kChains * 16384.0,
                          waves * kIters * 8 * 128.0, waves * kIters * 8 * 128.0};
    for (int k = 0; k < 4 && rc == 0; ++k) {
        for (int rep = 0; rep < 2 && rc == 0; ++rep) {   // the first launch loads the code object
            if (hipEventRecord(e0, s) != hipSuccess) rc = -4;
            if (k == 0) hipLaunchKernelGGL(k_peak_mfma64, dim3(blocks), dim3(256), 0, s, 1.0, out);
            if (k == 1) hipLaunchKernelGGL(k_peak_mfma16, dim3(blocks), dim3(256), 0, s, 0.5f, out);
            if (k == 2) hipLaunchKernelGGL(k_peak_fma<float>, dim3(blocks), dim3(256), 0, s, 1.0f, out);
            if (k == 3) hipLaunchKernelGGL(k_peak_fma<double>, dim3(blocks), dim3(256), 0, s, 1.0, out);
            if (hipGetLastError() != hipSuccess) rc = -4;
            if (rc == 0 && hipEventRecord(e1, s) != hipSuccess) rc = -4;
            if (rc == 0 && hipEventSynchronize(e1) != hipSuccess) rc = -4;
            float ms = 0.f;
            if (rc == 0 && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -4;
            if (rc == 0) tflops[k] = fl[k] / (ms * 1e-3) / 1e12;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(out);
    return rc;
}
