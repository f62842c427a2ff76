// Batched small dense kernels, one work-group per problem:
//  * shifted Cholesky of a Gram matrix (shifted CholeskyQR, Fukaya, Kannan,
//    Nakatsukasa, Zhang, Yamamoto, SIAM J. Sci. Comput. 2020),
//  * row-wise triangular solves Y <- Y R^-1,
//  * one-sided (Hestenes) Jacobi SVD of a k x k matrix,
// plus the blocked Cholesky / triangular solve of the dense diagonal tiles.
#include <algorithm>
#include <cmath>

#include "kernels.h"

namespace tlr {
namespace {

constexpr int kSmallThreads = 256;
constexpr int kLdsK = 124;  // k x k float64 (plus small arrays) fits in LDS up to this k
constexpr int kJacK = 112;  // Jacobi working copy k x (k+1) plus partial sums

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

__device__ inline double block_max(double v, double *red) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, red[w]);
    return t;
}

// ------------------------------------------------------ shifted Cholesky --

// In-place lower Cholesky of W (k x k, ld), left-looking by columns: for
// column c every row r >= c forms W[r][c] - sum_{q<c} L[r][q] L[c][q] (rows
// spread over the threads, two threads per row splitting the sum), then the
// column is scaled by the square root of its pivot.  A pivot <= defl
// (defl > 0) marks a dead direction: its whole column of L (so row of R,
// diagonal included) is zero, and the row solve writes a zero column of Q
// there.  Q keeps orthonormal live columns and Y = Q R still holds, so the
// singular values of R are those of Y.  Returns false on a non-positive or
// non-finite pivot when defl == 0 (uniform across the work-group).
__device__ bool chol_inplace(double *W, int ld, int k, double defl, double *part, int *s_fail) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int half = nt >> 1;  // threads [0, half) and [half, nt) split each row's sum
    const int side = tid / half, lt = tid - side * half;
    for (int c = 0; c < k; ++c) {
        const int qs = side ? (c >> 1) : 0, qe = side ? c : (c >> 1);
        for (int r = c + lt; r < k; r += half) {
            double acc = 0.0;
            for (int q = qs; q < qe; ++q) acc += W[r + q * ld] * W[c + q * ld];
            part[r + side * kMaxSketch] = acc;
        }
        __syncthreads();
        for (int r = c + tid; r < k; r += nt) part[r] = W[r + c * ld] - part[r] - part[r + kMaxSketch];
        __syncthreads();
        const double piv = part[c];
        if (!isfinite(piv) || (defl == 0.0 && !(piv > 0.0))) {
            if (tid == 0) *s_fail = c + 1;
            __syncthreads();
            return false;
        }
        if (defl > 0.0 && piv <= defl) {
            for (int r = c + tid; r < k; r += nt) W[r + c * ld] = 0.0;  // dead direction
        } else {
            const double inv = 1.0 / sqrt(piv);
            for (int r = c + tid; r < k; r += nt) W[r + c * ld] = (r == c) ? sqrt(piv) : part[r] * inv;
        }
        __syncthreads();
    }
    return true;
}

__global__ __launch_bounds__(kSmallThreads) void k_chol_small(const SmallDesc *__restrict__ descs,
                                                               int mode, DevParams *params) {
    __shared__ double lds[kLdsK * kLdsK];
    __shared__ double part[2 * kMaxSketch];
    __shared__ double red[kSmallThreads / 64];
    __shared__ int s_fail;
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    if (k <= 0) return;
    const int tid = threadIdx.x;
    double *W = (k <= kLdsK) ? lds : d.R;
    const int ldw = (k <= kLdsK) ? k : d.ldr;
    // mode 1: shifted (shift = 11 (m k + k (k+1)) u ||Y||^2, the squared norm
    // bounded by the trace);  mode 2: unshifted with deflation of pivots below
    // 1e-12 of the largest diagonal entry;  mode 0: plain.
    double shift = 0.0, defl = 0.0;
    if (mode == 1) {
        double tr = 0.0;
        for (int c = tid; c < k; c += blockDim.x) tr += d.A[c + (int64_t)c * d.lda];
        tr = block_sum(tr, red);
        shift = 11.0 * ((double)d.m * k + (double)k * (k + 1)) * 1.1102230246251565e-16 * tr;
        defl = 1e-300;  // an exactly-zero panel (zero tile) deflates instead of failing
    } else if (mode == 2) {
        double mx = 0.0;
        for (int c = tid; c < k; c += blockDim.x) mx = fmax(mx, d.A[c + (int64_t)c * d.lda]);
        mx = block_max(mx, red);
        defl = (mx > 0.0) ? 1e-12 * mx : 1e-300;
    }
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int r = e % k, q = e / k;
        if (r >= q) W[r + q * ldw] = d.A[r + (int64_t)q * d.lda] + ((r == q) ? shift : 0.0);
    }
    __syncthreads();
    const bool ok = chol_inplace(W, ldw, k, defl, part, &s_fail);
    if (!ok) {
        if (tid == 0) set_status(params, TLR_NOT_SPD, -100 - d.tile_i, -100 - d.tile_j);
        // leave an identity factor so downstream arithmetic stays finite
        for (int e = tid; e < k * k; e += blockDim.x) {
            const int r = e % k, q = e / k;
            d.R[r + (int64_t)q * d.ldr] = (r == q) ? 1.0 : 0.0;
        }
        return;
    }
    // R = L^T (upper), zero below the diagonal.  When W aliases R (k > kLdsK)
    // transpose in place through the upper triangle.
    if (W == d.R) {
        for (int e = tid; e < k * k; e += blockDim.x) {
            const int r = e % k, q = e / k;
            if (r > q) {
                W[q + r * ldw] = W[r + q * ldw];
            }
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += blockDim.x) {
            const int r = e % k, q = e / k;
            if (r > q) W[r + q * ldw] = 0.0;
        }
    } else {
        for (int e = tid; e < k * k; e += blockDim.x) {
            const int r = e % k, q = e / k;
            d.R[r + (int64_t)q * d.ldr] = (r <= q) ? W[q + r * ldw] : 0.0;
        }
    }
}

// ---------------------------------------------------------- row solves --

// Y (m x k) <- Y R^-1 for upper-triangular R.  A work-group of 64 threads
// owns 64 rows, held transposed in LDS (column c of the block is contiguous,
// so the 64 lanes read consecutive words); each thread runs the forward
// substitution of its row, 8 columns at a time in registers.  R is read with
// wave-uniform addresses.  Panels wider than kTrsmLds columns stay in global
// memory (same arithmetic).
constexpr int kTrsmLds = 240;

template <bool LDS>
__device__ void row_solve(double *yrow, int64_t stride, int k, const double *__restrict__ R, int64_t ldr) {
    constexpr int CH = 8;
    for (int c0 = 0; c0 < k; c0 += CH) {
        const int cw = (k - c0 < CH) ? (k - c0) : CH;
        double acc[CH];
#pragma unroll
        for (int t = 0; t < CH; ++t) acc[t] = (t < cw) ? yrow[(c0 + t) * stride] : 0.0;
        for (int q = 0; q < c0; ++q) {
            const double v = yrow[q * stride];
            const double *rq = R + q + c0 * ldr;
#pragma unroll
            for (int t = 0; t < CH; ++t)
                if (t < cw) acc[t] -= v * rq[t * ldr];
        }
#pragma unroll
        for (int t = 0; t < CH; ++t) {
            if (t < cw) {
                double a = acc[t];
#pragma unroll
                for (int tp = 0; tp < CH; ++tp)
                    if (tp < t) a -= acc[tp] * R[(c0 + tp) + (c0 + t) * ldr];
                const double rd = R[(c0 + t) + (c0 + t) * ldr];
                acc[t] = (rd != 0.0) ? a / rd : 0.0;  // zero diagonal: dead direction
            }
        }
#pragma unroll
        for (int t = 0; t < CH; ++t)
            if (t < cw) yrow[(c0 + t) * stride] = acc[t];
    }
}

__global__ __launch_bounds__(64) void k_trsm_rows(const SmallDesc *__restrict__ descs) {
    __shared__ double Yt[kTrsmLds * 64];
    const SmallDesc d = descs[blockIdx.y];
    const int k = d.k_dev ? *d.k_dev : d.k;
    const int r0 = blockIdx.x * 64;
    if (k <= 0 || r0 >= d.m) return;
    const int t = threadIdx.x;
    const int row = r0 + t;
    const bool valid = row < d.m;
    const int64_t ldy = d.ldy;
    if (k <= kTrsmLds) {
        for (int c = 0; c < k; ++c) Yt[c * 64 + t] = valid ? d.Y[row + c * ldy] : 0.0;
        row_solve<true>(Yt + t, 64, k, d.R, d.ldr);
        if (valid)
            for (int c = 0; c < k; ++c) d.Y[row + c * ldy] = Yt[c * 64 + t];
    } else if (valid) {
        row_solve<false>(d.Y + row, ldy, k, d.R, d.ldr);
    }
}

// ------------------------------------------------------ one-sided Jacobi --

// Rotates the columns of W (k x k, ld) until they are mutually orthogonal
// (one-sided Hestenes Jacobi).  Each round of the round-robin tournament
// pairs every column once; lane t of every wave owns pair t (t + 64, ...),
// and wave w owns the rows [w k/nw, (w+1) k/nw).  A round: every wave forms
// its partial inner products, one barrier, then each wave sums the partials of
// its pairs (all waves compute the same rotation) and rotates its own rows.
// Rows never cross waves, so the partial-product buffer is the only shared
// state (double-buffered across rounds).
__device__ void jacobi_columns(double *W, int ld, int k, double *part, int *s_rot) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6, nwaves = blockDim.x >> 6;
    const int kk = k + (k & 1);  // even player count; player k (odd k) sits out
    const int npairs = kk / 2;
    const int rlo = (k * wave) / nwaves, rhi = (k * (wave + 1)) / nwaves;
    const double eps = 1.0e-15 * sqrt((double)k);
    int buf = 0;
    for (int sweep = 0; sweep < 40; ++sweep) {
        if (tid == 0) *s_rot = 0;
        for (int round = 0; round < kk - 1; ++round) {
            double *pb = part + buf * (3 * kMaxSketch / 2 * 4);
            for (int pr = lane; pr < npairs; pr += 64) {
                const int a = (pr == 0) ? 0 : 1 + (pr - 1 + round) % (kk - 1);
                const int b = 1 + (kk - 2 - pr + round) % (kk - 1);
                double app = 0.0, aqq = 0.0, apq = 0.0;
                if (a < k && b < k) {
                    const int p = a < b ? a : b, q = a < b ? b : a;
                    const double *wp = W + (int64_t)p * ld, *wq = W + (int64_t)q * ld;
                    for (int r = rlo; r < rhi; ++r) {
                        const double x = wp[r], y = wq[r];
                        app += x * x;
                        aqq += y * y;
                        apq += x * y;
                    }
                }
                double *o = pb + (pr * nwaves + wave) * 3;
                o[0] = app;
                o[1] = aqq;
                o[2] = apq;
            }
            __syncthreads();
            bool any = false;
            for (int pr = lane; pr < npairs; pr += 64) {
                const int a = (pr == 0) ? 0 : 1 + (pr - 1 + round) % (kk - 1);
                const int b = 1 + (kk - 2 - pr + round) % (kk - 1);
                if (a >= k || b >= k) continue;
                double app = 0.0, aqq = 0.0, apq = 0.0;
                for (int w = 0; w < nwaves; ++w) {
                    const double *o = pb + (pr * nwaves + w) * 3;
                    app += o[0];
                    aqq += o[1];
                    apq += o[2];
                }
                if (apq != 0.0 && fabs(apq) > eps * sqrt(app * aqq)) {
                    const double zeta = (aqq - app) / (2.0 * apq);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
                    const int p = a < b ? a : b, q = a < b ? b : a;
                    double *wp = W + (int64_t)p * ld, *wq = W + (int64_t)q * ld;
                    for (int r = rlo; r < rhi; ++r) {
                        const double x = wp[r], y = wq[r];
                        wp[r] = cs * x - sn * y;
                        wq[r] = sn * x + cs * y;
                    }
                    any = true;
                }
            }
            if (any && wave == 0) *s_rot = 1;
            buf ^= 1;
        }
        __syncthreads();
        const int rot = *s_rot;
        __syncthreads();
        if (!rot) break;
    }
}

__global__ __launch_bounds__(kSmallThreads) void k_jacobi_svd(const SmallDesc *__restrict__ descs,
                                                               double tol, int min_tail, int k_full,
                                                               int rank_cap, DevParams *params) {
    __shared__ double lds[kJacK * (kJacK + 1)];
    __shared__ double s_norm[kMaxSketch];
    __shared__ int s_pos[kMaxSketch];
    __shared__ double part[2 * (3 * kMaxSketch / 2 * 4)];
    __shared__ int s_rot;
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    const int tid = threadIdx.x;
    if (k <= 0 || k > kMaxSketch) {
        if (tid == 0) {
            d.rank[0] = 0;
            d.rank[1] = 0;
            *d.flag = 0;
            if (k > kMaxSketch) set_status(params, TLR_RANK_OVERFLOW, d.tile_i, d.tile_j);
        }
        return;
    }
    // working copy: LDS for small k (odd pitch), else the caller's scratch d.R
    double *W = (k <= kJacK) ? lds : d.R;
    const int ldw = (k <= kJacK) ? k + 1 : d.ldr;
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int r = e % k, q = e / k;
        W[r + (int64_t)q * ldw] = d.A[r + (int64_t)q * d.lda];
    }
    __syncthreads();
    jacobi_columns(W, ldw, k, part, &s_rot);
    __syncthreads();
    for (int c = tid; c < k; c += blockDim.x) {
        double s2 = 0.0;
        for (int r = 0; r < k; ++r) {
            const double v = W[r + (int64_t)c * ldw];
            s2 += v * v;
        }
        s_norm[c] = sqrt(s2);
    }
    __syncthreads();
    for (int c = tid; c < k; c += blockDim.x) {
        const double sc = s_norm[c];
        int pos = 0;
        for (int q = 0; q < k; ++q) {
            const double sq = s_norm[q];
            pos += (sq > sc) || (sq == sc && q < c);
        }
        s_pos[c] = pos;
    }
    __syncthreads();
    // X[:, pos(c)] = W[:, c] / ||W[:, c]||, S[pos(c)] = ||W[:, c]||
    for (int e = tid; e < k * k; e += blockDim.x) {
        const int r = e % k, c = e / k;
        const double sc = s_norm[c];
        const double inv = (sc > 0.0) ? 1.0 / sc : 0.0;
        d.X[r + (int64_t)s_pos[c] * d.ldx] = W[r + (int64_t)c * ldw] * inv;
    }
    for (int c = tid; c < k; c += blockDim.x) d.S[s_pos[c]] = s_norm[c];
    __syncthreads();
    if (tid == 0) {
        int r = 0;
        for (int c = 0; c < k; ++c) r += (s_norm[c] > tol) ? 1 : 0;
        const int tail = k - r;
        const int insufficient = (tail < min_tail) && (k < (d.k_full < k_full ? d.k_full : k_full));
        int write = r;
        if (!insufficient && r > rank_cap) {
            set_status(params, TLR_RANK_OVERFLOW, d.tile_i, d.tile_j);
            write = rank_cap;
        }
        if (insufficient) write = 0;  // keep the previous factors; the host retries wider
        d.rank[0] = write;  // rank used to form the new factors
        d.rank[1] = r;      // numerical rank seen by this sample
        *d.flag = insufficient;
    }
}

// ------------------------------------------------- dense diagonal tiles --

// Cholesky of one bs x bs diagonal block A[b0:b0+bs, b0:b0+bs] (ld) in LDS.
__global__ __launch_bounds__(kSmallThreads) void k_potrf_block(double *A, int ld, int b0, int bs,
                                                                int tile, DevParams *params) {
    __shared__ double W[64 * 64];
    __shared__ double part[2 * kMaxSketch];
    __shared__ int s_fail;
    const int tid = threadIdx.x;
    if (params->status != 0) return;
    for (int e = tid; e < bs * bs; e += blockDim.x) {
        const int r = e % bs, q = e / bs;
        W[r + q * 64] = A[(b0 + r) + (int64_t)(b0 + q) * ld];
    }
    __syncthreads();
    const bool ok = chol_inplace(W, 64, bs, 0.0, part, &s_fail);
    if (!ok) {
        if (tid == 0) set_status(params, TLR_NOT_SPD, tile, tile);
        return;
    }
    for (int e = tid; e < bs * bs; e += blockDim.x) {
        const int r = e % bs, q = e / bs;
        if (r >= q) A[(b0 + r) + (int64_t)(b0 + q) * ld] = W[r + q * 64];
    }
}

// Rows r in [b0+bs, nrows): A[r, b0:b0+bs] <- A[r, b0:b0+bs] L_bb^-T.
__global__ __launch_bounds__(kSmallThreads) void k_potrf_panel(double *A, int ld, int b0, int bs,
                                                                int nrows, DevParams *params) {
    __shared__ double L[64 * 64];
    const int tid = threadIdx.x;
    if (params->status != 0) return;
    for (int e = tid; e < bs * bs; e += blockDim.x) {
        const int r = e % bs, q = e / bs;
        L[r + q * 64] = (r >= q) ? A[(b0 + r) + (int64_t)(b0 + q) * ld] : 0.0;
    }
    __syncthreads();
    const int row = b0 + bs + blockIdx.x * blockDim.x + tid;
    if (row >= nrows) return;
    double x[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) x[c] = (c < bs) ? A[row + (int64_t)(b0 + c) * ld] : 0.0;
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        if (c < bs) {
            double a = x[c];
            for (int cp = 0; cp < c; ++cp) a -= x[cp] * L[c + cp * 64];
            x[c] = a / L[c + c * 64];
        }
    }
#pragma unroll
    for (int c = 0; c < 64; ++c)
        if (c < bs) A[row + (int64_t)(b0 + c) * ld] = x[c];
}

// Panels B_t[b0:b0+bs, :] <- L_bb^-1 B_t[b0:b0+bs, :], one work-group per
// (panel, chunk of 64 columns); L_bb is the diagonal block of L (ld nb).
__global__ __launch_bounds__(64) void k_trsm_block(const double *__restrict__ L, int ldl, int b0, int bs,
                                                    const SmallDesc *__restrict__ descs) {
    __shared__ double Ls[64 * 64];
    const SmallDesc d = descs[blockIdx.y];
    const int cols = d.k_dev ? *d.k_dev : d.k;
    const int c = blockIdx.x * 64 + threadIdx.x;
    if (blockIdx.x * 64 >= cols) return;
    for (int e = threadIdx.x; e < bs * bs; e += 64) {
        const int r = e % bs, q = e / bs;
        Ls[r + q * 64] = (r >= q) ? L[(b0 + r) + (int64_t)(b0 + q) * ldl] : 0.0;
    }
    __syncthreads();
    if (c >= cols) return;
    double *y = d.Y + (int64_t)c * d.ldy + b0;
    double x[64];
#pragma unroll
    for (int r = 0; r < 64; ++r) x[r] = (r < bs) ? y[r] : 0.0;
#pragma unroll
    for (int r = 0; r < 64; ++r) {
        if (r < bs) {
            double a = x[r];
            for (int rp = 0; rp < r; ++rp) a -= Ls[r + rp * 64] * x[rp];
            x[r] = a / Ls[r + r * 64];
        }
    }
#pragma unroll
    for (int r = 0; r < 64; ++r)
        if (r < bs) y[r] = x[r];
}

}  // namespace

tlr_status chol_small(const SmallDesc *d_descs, int count, int max_k, int mode, DevParams *params,
                      hipStream_t s) {
    (void)max_k;
    if (count <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_chol_small, dim3(count), dim3(kSmallThreads), 0, s, d_descs, mode, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status trsm_rows(const SmallDesc *d_descs, int count, int max_m, int max_k, hipStream_t s) {
    (void)max_k;
    if (count <= 0 || max_m <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_trsm_rows, dim3((unsigned)cdiv(max_m, 64), count), dim3(64), 0, s, d_descs);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status jacobi_svd(const SmallDesc *d_descs, int count, int max_k, double tol, int min_tail,
                      int k_full, int rank_cap, DevParams *params, hipStream_t s) {
    (void)max_k;
    if (count <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_jacobi_svd, dim3(count), dim3(kSmallThreads), 0, s, d_descs, tol, min_tail,
                       k_full, rank_cap, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

void potrf_tile_descs(double *A, int nb, GemmDesc *h) {
    const int nblk = (int)cdiv(nb, 64);
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        GemmDesc g{};
        g.A = A + (b0 + bs) + (int64_t)b0 * nb;
        g.B = A + (b0 + bs) + (int64_t)b0 * nb;
        g.C = A + (b0 + bs) + (int64_t)(b0 + bs) * nb;
        g.M = rest;
        g.N = rest;
        g.K = bs;
        g.lda = nb;
        g.ldb = nb;
        g.ldc = nb;
        g.alpha = -1.0;
        g.beta = 1.0;
        h[b] = g;
    }
}

tlr_status potrf_tile(double *A, int nb, int tile, DevParams *params, const GemmDesc *d_desc, hipStream_t s) {
    const int nblk = (int)cdiv(nb, 64);
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(kSmallThreads), 0, s, A, nb, b0, bs, tile, params);
        if (rest > 0) {
            hipLaunchKernelGGL(k_potrf_panel, dim3((unsigned)cdiv(rest, kSmallThreads)),
                               dim3(kSmallThreads), 0, s, A, nb, b0, bs, nb, params);
            TLR_TRY(gemm_batched(false, true, d_desc + b, 1, rest, rest, s));
        }
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

namespace {
__global__ void k_copy_batched(const CopyDesc *__restrict__ descs) {
    const CopyDesc d = descs[blockIdx.y];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.words;
         e += (int64_t)gridDim.x * blockDim.x)
        d.dst[e] = d.src[e];
}
}  // namespace

tlr_status copy_batched(const CopyDesc *d_descs, int count, int64_t max_words, hipStream_t s) {
    if (count <= 0 || max_words <= 0) return TLR_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(max_words, 256), 256);
    hipLaunchKernelGGL(k_copy_batched, dim3(gx, count), dim3(256), 0, s, d_descs);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status trsm_left_lower(const double *L, int nb, const SmallDesc *d_descs, const SmallDesc *h_descs,
                           int count, int max_cols, GemmDesc *d_gemm, GemmDesc *h_gemm, hipStream_t s) {
    if (count <= 0 || max_cols <= 0) return TLR_OK;
    const int nblk = (int)cdiv(nb, 64);
    // block b, panel t: Y_t[b0+bs:, :] -= L[b0+bs:, b0:b0+bs] * Y_t[b0:b0+bs, :]
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        for (int t = 0; t < count; ++t) {
            const SmallDesc &pd = h_descs[t];
            GemmDesc o{};
            o.A = L + (b0 + bs) + (int64_t)b0 * nb;
            o.lda = nb;
            o.B = pd.Y + b0;
            o.ldb = pd.ldy;
            o.C = pd.Y + b0 + bs;
            o.ldc = pd.ldy;
            o.M = rest;
            o.N = pd.k;
            o.N_dev = pd.k_dev;
            o.K = bs;
            o.alpha = -1.0;
            o.beta = 1.0;
            h_gemm[(int64_t)b * count + t] = o;
        }
    }
    TLR_HIP(hipMemcpyAsync(d_gemm, h_gemm, sizeof(GemmDesc) * count * nblk, hipMemcpyHostToDevice, s));
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        hipLaunchKernelGGL(k_trsm_block, dim3((unsigned)cdiv(max_cols, 64), count), dim3(64), 0, s, L, nb,
                           b0, bs, d_descs);
        if (rest > 0)
            TLR_TRY(gemm_batched(false, false, d_gemm + (int64_t)b * count, count, rest, max_cols, s));
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
