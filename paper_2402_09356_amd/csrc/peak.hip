// Attainable-peak probes of the two roofs the likelihood path is measured
// against: HBM bandwidth (a streaming copy) and FP64 matrix-core throughput
// (a loop of independent v_mfma_f64_16x16x4 chains).  Each is timed with HIP
// events on the caller's stream; the roofline fractions of the benchmark are
// taken against these measured figures as well as against the published ones.
#include <algorithm>

#include "kernels.h"

namespace tlr {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

// dst = src over `n16` 16-byte words: each thread moves four words a pass,
// all four loads in flight before the stores; the grid strides over the
// buffer so that every compute unit streams.
__global__ __launch_bounds__(256) void k_peak_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   int64_t n16) {
    const int64_t stride = (int64_t)gridDim.x * 256 * 4;
    for (int64_t base = (int64_t)blockIdx.x * 256 * 4 + threadIdx.x; base < n16; base += stride) {
        double2 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = base + 256 * u;
            if (e < n16) v[u] = src[e];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t e = base + 256 * u;
            if (e < n16) dst[e] = v[u];
        }
    }
}

// Eight independent accumulator chains a wave (enough to cover the MFMA
// pipeline), `iters` steps each; the sums are stored so nothing is elided.
__global__ __launch_bounds__(256) void k_peak_mfma_f64(double *out, int iters, double seed) {
    const int lane = threadIdx.x & 63;
    double a = seed + 1e-3 * lane, b = 1.0 - 1e-3 * lane;
    v4d acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = v4d{0.0, 0.0, 0.0, 0.0};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int c = 0; c < 8; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
    }
    v4d s = acc[0];
#pragma unroll
    for (int c = 1; c < 8; ++c) s += acc[c];
    const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
    out[t] = s[0] + s[1] + s[2] + s[3];
}

}  // namespace

tlr_status peak_hbm(const void *src, void *dst, int64_t bytes, int reps, double *gbs, hipStream_t s) {
    if (!src || !dst || bytes < 16 || reps < 1 || !gbs) return TLR_E_INVAL;
    const int64_t n16 = bytes / 16;
    int dev = 0, cus = 0;
    TLR_HIP(hipGetDevice(&dev));
    TLR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const unsigned grid = (unsigned)std::max(1, cus * 8);
    hipEvent_t e0, e1;
    TLR_HIP(hipEventCreate(&e0));
    TLR_HIP(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_peak_copy, dim3(grid), dim3(256), 0, s, static_cast<const double2 *>(src),
                       static_cast<double2 *>(dst), n16);  // warm
    TLR_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r)
        hipLaunchKernelGGL(k_peak_copy, dim3(grid), dim3(256), 0, s, static_cast<const double2 *>(src),
                           static_cast<double2 *>(dst), n16);
    TLR_HIP(hipEventRecord(e1, s));
    TLR_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TLR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // every byte read once and written once
    *gbs = 2.0 * 16.0 * (double)n16 * reps / (ms * 1e-3) / 1e9;
    return TLR_OK;
}

tlr_status peak_mfma_f64(double *scratch, int64_t scratch_words, int iters, double *tflops, hipStream_t s) {
    if (!scratch || iters < 1 || !tflops) return TLR_E_INVAL;
    int dev = 0, cus = 0;
    TLR_HIP(hipGetDevice(&dev));
    TLR_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // eight waves a compute unit: two on each SIMD
    const int64_t grid = (int64_t)cus * 2;
    if (scratch_words < grid * 256) return TLR_E_NOMEM;
    hipEvent_t e0, e1;
    TLR_HIP(hipEventCreate(&e0));
    TLR_HIP(hipEventCreate(&e1));
    hipLaunchKernelGGL(k_peak_mfma_f64, dim3((unsigned)grid), dim3(256), 0, s, scratch, 16, 0.5);  // warm
    TLR_HIP(hipEventRecord(e0, s));
    hipLaunchKernelGGL(k_peak_mfma_f64, dim3((unsigned)grid), dim3(256), 0, s, scratch, iters, 0.5);
    TLR_HIP(hipEventRecord(e1, s));
    TLR_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    TLR_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const double waves = (double)grid * 4.0;
    const double flops = waves * iters * 8.0 * (16.0 * 16.0 * 4.0 * 2.0);
    *tflops = flops / (ms * 1e-3) / 1e12;
    return TLR_OK;
}

}  // namespace tlr
