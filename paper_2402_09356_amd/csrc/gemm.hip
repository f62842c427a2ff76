// Batched float64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// Each work-group computes a 64 x 64 block of one product of the batch with
// four waves in a 2 x 2 arrangement (32 x 32 per wave = 2 x 2 MFMA tiles of
// 16 x 16).  A and B stream through LDS in K-slices of 16, stored k-major so
// that the 16 lanes reading one MFMA operand column touch consecutive words.
// Sizes are per product (possibly device-resident); work-groups whose block
// lies outside their product exit at once, so the grid is sized by the
// largest product.
#include "kernels.h"
#include "ktimer.h"

namespace tlr {
namespace {

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int PADM = BM + 4;  // LDS row pitch (doubles) to spread banks
constexpr int PADN = BN + 4;

typedef double v4d __attribute__((ext_vector_type(4)));

template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm_f64(const GemmDesc *__restrict__ descs, int tiles_n) {
    const GemmDesc d = descs[blockIdx.y];
    const int M = d.M_dev ? *d.M_dev : d.M;
    const int N = d.N_dev ? *d.N_dev : d.N;
    const int K = d.K_dev ? *d.K_dev : d.K;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= M || n0 >= N) return;

    __shared__ double As[BK][PADM];
    __shared__ double Bs[BK][PADN];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;
    const int li = lane & 15, lk = lane >> 4;

    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    const double *__restrict__ A = d.A;
    const double *__restrict__ B = d.B;
    const int64_t lda = d.lda, ldb = d.ldb;

    for (int k0 = 0; k0 < K; k0 += BK) {
        // A slice: BM x BK elements of op(A)
#pragma unroll
        for (int r = 0; r < (BM * BK) / 256; ++r) {
            const int e = tid + r * 256;
            int mm, kk;
            if (!TA) {
                mm = e % BM;
                kk = e / BM;
            } else {
                kk = e % BK;
                mm = e / BK;
            }
            const int gm = m0 + mm, gk = k0 + kk;
            double v = 0.0;
            if (gm < M && gk < K) v = TA ? A[gk + gm * lda] : A[gm + gk * lda];
            As[kk][mm] = v;
        }
        // B slice: BK x BN elements of op(B)
#pragma unroll
        for (int r = 0; r < (BN * BK) / 256; ++r) {
            const int e = tid + r * 256;
            int kk, nn;
            if (!TB) {
                kk = e % BK;
                nn = e / BK;
            } else {
                nn = e % BN;
                kk = e / BN;
            }
            const int gn = n0 + nn, gk = k0 + kk;
            double v = 0.0;
            if (gn < N && gk < K) v = TB ? B[gn + gk * ldb] : B[gk + gn * ldb];
            Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int ks = 0; ks < BK; ks += 4) {
            double a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i) a[i] = As[ks + lk][wm + i * 16 + li];
#pragma unroll
            for (int j = 0; j < 2; ++j) b[j] = Bs[ks + lk][wn + j * 16 + li];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        __syncthreads();
    }

    // D layout of the 16x16 f64 MFMA (measured on gfx950): lane holds column
    // (lane % 16); its register r holds row (lane / 16) + 4 r.
    double *__restrict__ C = d.C;
    const int64_t ldc = d.ldc;
    const double alpha = d.alpha, beta = d.beta;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int gn = n0 + wn + j * 16 + li;
            if (gn >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm + i * 16 + lk + 4 * r;
                if (gm >= M) continue;
                double *c = C + gm + gn * ldc;
                const double v = alpha * acc[i][j][r];
                *c = (beta == 0.0) ? v : v + beta * (*c);
            }
        }
}

}  // namespace

tlr_status gemm_batched(bool trans_a, bool trans_b, const GemmDesc *d_descs, int count, int max_m,
                        int max_n, hipStream_t s, const GemmDesc *h_descs) {
    if (count <= 0 || max_m <= 0 || max_n <= 0) return TLR_OK;
    const int tiles_m = (int)cdiv(max_m, BM), tiles_n = (int)cdiv(max_n, BN);
    if (count > 65535) return TLR_E_UNSUPPORTED;
    static const int cls[4] = {ktimer_class("k_gemm_f64<N,N>"), ktimer_class("k_gemm_f64<N,T>"),
                               ktimer_class("k_gemm_f64<T,N>"), ktimer_class("k_gemm_f64<T,T>")};
    double flops = 0.0, bytes = 0.0;
    bool exact = h_descs != nullptr;
    if (exact && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const GemmDesc &g = h_descs[t];
            if (g.M_dev || g.N_dev || g.K_dev) exact = false;
            const double M = g.M, N = g.N, K = g.K;
            flops += 2.0 * M * N * K;
            bytes += 8.0 * (M * K + K * N + M * N * (g.beta != 0.0 ? 2.0 : 1.0));
        }
    KTimer kt(cls[(trans_a ? 2 : 0) + (trans_b ? 1 : 0)], s, flops, bytes, exact);
    const dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)count), block(256);
    if (!trans_a && !trans_b)
        hipLaunchKernelGGL((k_gemm_f64<false, false>), grid, block, 0, s, d_descs, tiles_n);
    else if (!trans_a && trans_b)
        hipLaunchKernelGGL((k_gemm_f64<false, true>), grid, block, 0, s, d_descs, tiles_n);
    else if (trans_a && !trans_b)
        hipLaunchKernelGGL((k_gemm_f64<true, false>), grid, block, 0, s, d_descs, tiles_n);
    else
        hipLaunchKernelGGL((k_gemm_f64<true, true>), grid, block, 0, s, d_descs, tiles_n);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
