// Batched float64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64).
//
// The products here are skinny: K is a tile edge (hundreds) while M x N is a
// sketch or a Gram matrix (tens to a few hundred).  A work-group owns one
// 32 x 32 block of C; its four waves split K (16-wide slices, wave w takes
// slices w, w+4, ...) and each computes the whole block over its slices
// (2 x 2 MFMA tiles), reading its operands straight from global memory in
// MFMA operand layout, one slice ahead of the arithmetic.  The four partial
// blocks meet once in LDS and are summed in a fixed order (deterministic).
// Sizes are per product (possibly device-resident); work-groups whose block
// lies outside their product exit at once, so the grid is sized by the
// largest product.
//
// Element types: each operand and the result may be float64 or float32 (the
// factors of the mixed-precision path are stored in float32).  A float32
// operand is widened to float64 as it is loaded and the product is formed and
// accumulated in float64 on the matrix cores; a float32 result is rounded once
// when it is stored.
#include "kernels.h"
#include "ktimer.h"

namespace tlr {
namespace {

constexpr int BM = 32, BN = 32, BK = 16;
// a product batch is "tall" (streaming kernels) from this many rows of C and
// this many 64-row blocks over the batch
constexpr int kTallM = 256, kTallBlocks = 256;

typedef double v4d __attribute__((ext_vector_type(4)));

// One 16-deep slice of both operands in their stored element types: a
// float32 value is widened only where the matrix core consumes it, so the
// next slice's loads stay in flight across the current slice's arithmetic.
template <class EA, class EB>
struct Slice {
    EA a[4][2];  // [k step][tile]
    EB b[4][2];
};

template <bool TA, bool TB, class EA, class EB>
__device__ inline void load_slice(Slice<EA, EB> &sl, const EA *__restrict__ A, int64_t lda, const EB *__restrict__ B,
                                  int64_t ldb, int m0, int n0, int k0, int M, int N, int K, int li, int lk) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int kk = k0 + 4 * t + lk;
        const bool kin = kk < K;
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const int r = m0 + 16 * i + li;
            sl.a[t][i] = (kin && r < M) ? (TA ? A[kk + r * lda] : A[r + kk * lda]) : EA(0);
        }
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int c = n0 + 16 * j + li;
            sl.b[t][j] = (kin && c < N) ? (TB ? B[c + kk * ldb] : B[kk + c * ldb]) : EB(0);
        }
    }
}

// lower_only: blocks wholly above the diagonal are skipped (products whose
// consumer reads only the lower triangle: Gram matrices, symmetric updates).
// NW waves split K (four, or eight for the Gram matrices, whose K is the
// long tile edge and whose blocks are few).
template <bool TA, bool TB, int NW, class EA, class EB, class EC>
__global__ __launch_bounds__(NW * 64) void k_gemm_f64(const GemmDesc *descs, int tiles_n, int lower_only) {
    const GemmDesc d = descs[blockIdx.y];
    const int M = d.M_dev ? *d.M_dev : d.M;
    const int N = d.N_dev ? *d.N_dev : d.N;
    const int K = d.K_dev ? *d.K_dev : d.K;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= M || n0 >= N || (lower_only && n0 > m0)) return;

    __shared__ double red[NW][BM * BN];

    const int tid = threadIdx.x;
    const int wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const EA *__restrict__ A = static_cast<const EA *>(d.A);
    const EB *__restrict__ B = static_cast<const EB *>(d.B);
    const int64_t lda = d.lda, ldb = d.ldb;

    v4d acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    const int nsl = (K + BK - 1) / BK;
    Slice<EA, EB> cur, nxt;
    if (wave < nsl) load_slice<TA, TB, EA, EB>(cur, A, lda, B, ldb, m0, n0, wave * BK, M, N, K, li, lk);
    for (int s = wave; s < nsl; s += NW) {
        if (s + NW < nsl) load_slice<TA, TB, EA, EB>(nxt, A, lda, B, ldb, m0, n0, (s + NW) * BK, M, N, K, li, lk);
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64((double)cur.a[t][i], (double)cur.b[t][j],
                                                                     acc[i][j], 0, 0, 0);
        cur = nxt;
    }

    // D layout of the 16x16 f64 MFMA (measured on gfx950): lane holds column
    // (lane % 16); its register r holds row (lane / 16) + 4 r.
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave][(16 * i + lk + 4 * r) + BM * (16 * j + li)] = acc[i][j][r];
    __syncthreads();
    EC *__restrict__ C = static_cast<EC *>(d.C);
    const int64_t ldc = d.ldc;
    const double alpha = d.alpha, beta = d.beta;
#pragma unroll
    for (int e = tid; e < BM * BN; e += NW * 64) {
        const int r = e % BM, c = e / BM;
        const int gm = m0 + r, gn = n0 + c;
        if (gm < M && gn < N) {
            double sum = red[0][e];
#pragma unroll
            for (int w = 1; w < NW; ++w) sum += red[w][e];
            const double v = alpha * sum;
            EC *cp = C + gm + gn * ldc;
            *cp = (EC)((beta == 0.0) ? v : v + beta * (double)(*cp));
        }
    }
}

// Tall products with a wider right factor, or a transposed left one: a
// work-group owns a BM x BN block of C, its four waves a 2 x 2 grid of
// (BM/2) x (BN/2) blocks over the whole of K.  Each 16-deep slice of op(A)
// and op(B) is read coalesced (along whichever index is contiguous in
// memory) into registers one slice ahead, then stored k-major in LDS, where
// the waves read their MFMA operands.
template <bool TA, bool TB, int BM, int BN, class EA, class EB, class EC>
__global__ __launch_bounds__(256) void k_gemm_lds(const GemmDesc *descs, int tiles_n) {
    constexpr int BK = 16, TM = BM / 32, TN = BN / 32;
    constexpr int PA = BM + 1, PB = BN + 1;
    constexpr int LA = BM * BK / 256, LB = BN * BK / 256;
    const GemmDesc d = descs[blockIdx.y];
    const int M = d.M_dev ? *d.M_dev : d.M;
    const int N = d.N_dev ? *d.N_dev : d.N;
    const int K = d.K_dev ? *d.K_dev : d.K;
    const int tm = blockIdx.x / tiles_n, tn = blockIdx.x % tiles_n;
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= M || n0 >= N) return;
    __shared__ double As[2][BK * PA];
    __shared__ double Bs[2][BK * PB];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int li = lane & 15, lk = lane >> 4;
    const int wm = wave >> 1, wn = wave & 1;
    const EA *__restrict__ A = static_cast<const EA *>(d.A);
    const EB *__restrict__ B = static_cast<const EB *>(d.B);
    const int64_t lda = d.lda, ldb = d.ldb;
    EA ra[LA];  // stored types: widened when written to LDS, after the slice's arithmetic
    EB rb[LB];
    auto gload = [&](int k0) {
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const int e = tid + 256 * u;
            const int m = TA ? e / BK : e % BM, k = TA ? e % BK : e / BM;
            const int gm = m0 + m, gk = k0 + k;
            ra[u] = (gm < M && gk < K) ? (TA ? A[gk + gm * lda] : A[gm + gk * lda]) : EA(0);
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = tid + 256 * u;
            const int n = TB ? e % BN : e / BK, k = TB ? e / BN : e % BK;
            const int gn = n0 + n, gk = k0 + k;
            rb[u] = (gn < N && gk < K) ? (TB ? B[gn + gk * ldb] : B[gk + gn * ldb]) : EB(0);
        }
    };
    auto lstore = [&](int buf) {
#pragma unroll
        for (int u = 0; u < LA; ++u) {
            const int e = tid + 256 * u;
            const int m = TA ? e / BK : e % BM, k = TA ? e % BK : e / BM;
            As[buf][k * PA + m] = (double)ra[u];
        }
#pragma unroll
        for (int u = 0; u < LB; ++u) {
            const int e = tid + 256 * u;
            const int n = TB ? e % BN : e / BK, k = TB ? e / BN : e % BK;
            Bs[buf][k * PB + n] = (double)rb[u];
        }
    };
    v4d acc[TM][TN];
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
    const int nsl = (K + BK - 1) / BK;
    gload(0);
    lstore(0);
    __syncthreads();
    for (int sl = 0; sl < nsl; ++sl) {
        const int buf = sl & 1;
        if (sl + 1 < nsl) gload((sl + 1) * BK);
        const double *as = As[buf], *bs = Bs[buf];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            double av[TM], bv[TN];
#pragma unroll
            for (int i = 0; i < TM; ++i) av[i] = as[(4 * t + lk) * PA + wm * (BM / 2) + 16 * i + li];
#pragma unroll
            for (int j = 0; j < TN; ++j) bv[j] = bs[(4 * t + lk) * PB + wn * (BN / 2) + 16 * j + li];
#pragma unroll
            for (int i = 0; i < TM; ++i)
#pragma unroll
                for (int j = 0; j < TN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
        }
        if (sl + 1 < nsl) lstore(buf ^ 1);
        __syncthreads();
    }
    EC *__restrict__ C = static_cast<EC *>(d.C);
    const int64_t ldc = d.ldc;
    const double alpha = d.alpha, beta = d.beta;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int gm = m0 + wm * (BM / 2) + 16 * i + lk + 4 * r;
                const int gn = n0 + wn * (BN / 2) + 16 * j + li;
                if (gm < M && gn < N) {
                    EC *cp = C + gm + (int64_t)gn * ldc;
                    const double v = alpha * acc[i][j][r];
                    *cp = (EC)((beta == 0.0) ? v : v + beta * (double)(*cp));
                }
            }
}


// Launch one batch with element types (EA, EB, EC).
template <class EA, class EB, class EC>
tlr_status launch_typed(bool trans_a, bool trans_b, const GemmDesc *d_descs, int count, int max_m, int max_n,
                        hipStream_t s, double flops, double bytes, bool exact, bool lower_only) {
    const int tiles_m = (int)cdiv(max_m, BM), tiles_n = (int)cdiv(max_n, BN);
    static const int cls[4] = {ktimer_class("k_gemm_f64<N,N>"), ktimer_class("k_gemm_f64<N,T>"),
                               ktimer_class("k_gemm_f64<T,N>"), ktimer_class("k_gemm_f64<T,T>")};
    // tall products (many rows of C) go to the LDS-staged kernel, which reads
    // both operands along their contiguous index and needs no final
    // reduction: 64 x 64 blocks for a right factor of 33..64 columns, else
    // 64 x 32; short ones keep the K-split kernel, which spreads a long K over
    // four waves (Gram matrices, small sketches)
    const int row_blocks = (int)cdiv(max_m, 64);
    if (!lower_only && !trans_b && max_m >= kTallM && (int64_t)row_blocks * count >= kTallBlocks) {
        static const int cls_t = ktimer_class("k_gemm_lds<T,N>"), cls_w = ktimer_class("k_gemm_lds<N,N>");
        KTimer kt(trans_a ? cls_t : cls_w, s, flops, bytes, exact);
        if (max_n > 32 && (trans_a || max_n <= 64)) {
            const int tn = (int)cdiv(max_n, 64);
            const dim3 grid((unsigned)(row_blocks * tn), (unsigned)count);
            if (trans_a)
                hipLaunchKernelGGL((k_gemm_lds<true, false, 64, 64, EA, EB, EC>), grid, dim3(256), 0, s, d_descs, tn);
            else
                hipLaunchKernelGGL((k_gemm_lds<false, false, 64, 64, EA, EB, EC>), grid, dim3(256), 0, s, d_descs,
                                   tn);
        } else {
            const int tn = (int)cdiv(max_n, 32);
            const dim3 grid((unsigned)(row_blocks * tn), (unsigned)count);
            if (trans_a)
                hipLaunchKernelGGL((k_gemm_lds<true, false, 64, 32, EA, EB, EC>), grid, dim3(256), 0, s, d_descs, tn);
            else
                hipLaunchKernelGGL((k_gemm_lds<false, false, 64, 32, EA, EB, EC>), grid, dim3(256), 0, s, d_descs,
                                   tn);
        }
        TLR_HIP(hipGetLastError());
        return TLR_OK;
    }
    KTimer kt(cls[(trans_a ? 2 : 0) + (trans_b ? 1 : 0)], s, flops, bytes, exact);
    const dim3 grid((unsigned)(tiles_m * tiles_n), (unsigned)count);
    const int lo = lower_only ? 1 : 0;
    if (lower_only) {
        const dim3 block(512);
        if (!trans_a && !trans_b)
            hipLaunchKernelGGL((k_gemm_f64<false, false, 8, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else if (!trans_a && trans_b)
            hipLaunchKernelGGL((k_gemm_f64<false, true, 8, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else if (trans_a && !trans_b)
            hipLaunchKernelGGL((k_gemm_f64<true, false, 8, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else
            hipLaunchKernelGGL((k_gemm_f64<true, true, 8, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
    } else {
        const dim3 block(256);
        if (!trans_a && !trans_b)
            hipLaunchKernelGGL((k_gemm_f64<false, false, 4, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else if (!trans_a && trans_b)
            hipLaunchKernelGGL((k_gemm_f64<false, true, 4, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else if (trans_a && !trans_b)
            hipLaunchKernelGGL((k_gemm_f64<true, false, 4, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
        else
            hipLaunchKernelGGL((k_gemm_f64<true, true, 4, EA, EB, EC>), grid, block, 0, s, d_descs, tiles_n, lo);
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace

tlr_status gemm_batched(bool trans_a, bool trans_b, const GemmDesc *d_descs, int count, int max_m,
                        int max_n, hipStream_t s, const GemmDesc *h_descs, bool lower_only, int types) {
    if (count <= 0 || max_m <= 0 || max_n <= 0) return TLR_OK;
    if (count > 65535) return TLR_E_UNSUPPORTED;
    const double wa = (types & kGemmA32) ? 4.0 : 8.0, wb = (types & kGemmB32) ? 4.0 : 8.0,
                 wc = (types & kGemmC32) ? 4.0 : 8.0;
    double flops = 0.0, bytes = 0.0;
    bool exact = h_descs != nullptr;
    if (exact && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const GemmDesc &g = h_descs[t];
            if (g.M_dev || g.N_dev || g.K_dev) exact = false;
            const double M = g.M, N = g.N, K = g.K;
            // a lower-only product computes the M(M+1)/2 entries on and below
            // the diagonal (M = N for every such product here)
            const double outs = lower_only ? M * (M + 1.0) / 2.0 : M * N;
            flops += 2.0 * outs * K;
            bytes += wa * M * K + wb * K * N + wc * outs * (g.beta != 0.0 ? 2.0 : 1.0);
        }
    switch (types) {
        case 0:
            return launch_typed<double, double, double>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                        bytes, exact, lower_only);
        case kGemmC32:
            return launch_typed<double, double, float>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                       bytes, exact, lower_only);
        case kGemmA32:
            return launch_typed<float, double, double>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                       bytes, exact, lower_only);
        case kGemmA32 | kGemmB32:
            return launch_typed<float, float, double>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                      bytes, exact, lower_only);
        case kGemmA32 | kGemmC32:
            return launch_typed<float, double, float>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                      bytes, exact, lower_only);
        case kGemmB32 | kGemmC32:
            return launch_typed<double, float, float>(trans_a, trans_b, d_descs, count, max_m, max_n, s, flops,
                                                      bytes, exact, lower_only);
        default:
            return TLR_E_UNSUPPORTED;
    }
}

}  // namespace tlr
