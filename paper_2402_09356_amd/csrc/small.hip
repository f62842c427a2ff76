// Batched small dense kernels, one work-group per problem:
//  * shifted Cholesky of a Gram matrix (shifted CholeskyQR, Fukaya, Kannan,
//    Nakatsukasa, Zhang, Yamamoto, SIAM J. Sci. Comput. 2020),
//  * row-wise triangular solves Y <- Y R^-1,
//  * one-sided (Hestenes) Jacobi SVD of a k x k matrix,
// plus the blocked Cholesky / triangular solve of the dense diagonal tiles.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "ktimer.h"

namespace tlr {
namespace {

constexpr int kSmallThreads = 256;
constexpr int kLdsK = 124;  // k x k float64 (plus small arrays) fits in LDS up to this k
constexpr int kJacK = 112;  // Jacobi working copy k x (k+1) plus partial sums
constexpr int kPackK = 176; // packed lower triangle k(k+1)/2 <= kLdsK^2 doubles
constexpr int kRegK = 176;  // register-resident pivoted QR (one column per thread)
constexpr int kCholLds = (kLdsK * kLdsK > kPackK * (kPackK + 1) / 2) ? kLdsK * kLdsK : kPackK * (kPackK + 1) / 2;
static_assert(kPackK * (kPackK + 1) / 2 <= kCholLds, "packed Cholesky must fit its LDS array");

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

// Cholesky of W (k x k, global, ld) in 64-wide blocks, right-looking: the
// diagonal block is factored in LDS, the panel below is solved row by row
// against it in place, and the trailing lower triangle is updated from the
// panel (all in global memory, which stays in L2 at these sizes).  For k too
// large to hold W in LDS.  Same deflation rule as chol_inplace.
__device__ bool chol_blocked_global(double *W, int ld, int k, double defl, double *Lb, double *part, int *s_fail) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int b0 = 0; b0 < k; b0 += 64) {
        const int bs = (k - b0 < 64) ? k - b0 : 64;
        for (int e = tid; e < 64 * 64; e += nt) {
            const int r = e & 63, q = e >> 6;
            Lb[e] = (r < bs && q < bs) ? W[(b0 + r) + (int64_t)(b0 + q) * ld] : 0.0;
        }
        __syncthreads();
        if (!chol_inplace(Lb, 64, bs, defl, part, s_fail)) return false;
        for (int e = tid; e < 64 * 64; e += nt) {
            const int r = e & 63, q = e >> 6;
            if (r < bs && q < bs && r >= q) W[(b0 + r) + (int64_t)(b0 + q) * ld] = Lb[r + q * 64];
        }
        const int rest = k - b0 - bs;
        if (rest <= 0) break;
        // panel rows: x L_bb^T = a  (a dead diagonal gives a zero entry)
        for (int rr = tid; rr < rest; rr += nt) {
            double *wr = W + (b0 + bs + rr) + (int64_t)b0 * ld;
            for (int cc = 0; cc < bs; ++cc) {
                double a = wr[(int64_t)cc * ld];
                for (int cp = 0; cp < cc; ++cp) a -= wr[(int64_t)cp * ld] * Lb[cc + cp * 64];
                const double dg = Lb[cc + cc * 64];
                wr[(int64_t)cc * ld] = (dg != 0.0) ? a / dg : 0.0;
            }
        }
        __syncthreads();
        // trailing lower triangle: W[r][q] -= sum_c P[r][c] P[q][c]
        for (int e = tid; e < rest * rest; e += nt) {
            const int rr = e % rest, qq = e / rest;
            if (rr < qq) continue;
            const double *pr = W + (b0 + bs + rr) + (int64_t)b0 * ld;
            const double *pq = W + (b0 + bs + qq) + (int64_t)b0 * ld;
            double acc = 0.0;
            for (int cc = 0; cc < bs; ++cc) acc += pr[(int64_t)cc * ld] * pq[(int64_t)cc * ld];
            W[(b0 + bs + rr) + (int64_t)(b0 + bs + qq) * ld] -= acc;
        }
        __syncthreads();
    }
    return true;
}

// Lower Cholesky with the lower triangle packed by columns in LDS: (r, q),
// r >= q, at q*k - q(q-1)/2 + (r - q).  Same algorithm and deflation rule as
// chol_inplace; lets k up to kPackK stay on chip.
__device__ inline int pk(int r, int q, int k) { return q * k - (q * (q - 1)) / 2 + (r - q); }

__device__ bool chol_packed(double *P, int k, double defl, double *part, int *s_fail) {
    const int tid = threadIdx.x, nt = blockDim.x;
    const int half = nt >> 1;
    const int side = tid / half, lt = tid - side * half;
    for (int c = 0; c < k; ++c) {
        const int qs = side ? (c >> 1) : 0, qe = side ? c : (c >> 1);
        for (int r = c + lt; r < k; r += half) {
            double acc = 0.0;
            for (int q = qs; q < qe; ++q) acc += P[pk(r, q, k)] * P[pk(c, q, k)];
            part[r + side * kMaxSketch] = acc;
        }
        __syncthreads();
        for (int r = c + tid; r < k; r += nt) part[r] = P[pk(r, c, k)] - part[r] - part[r + kMaxSketch];
        __syncthreads();
        const double piv = part[c];
        if (!isfinite(piv) || (defl == 0.0 && !(piv > 0.0))) {
            if (tid == 0) *s_fail = c + 1;
            __syncthreads();
            return false;
        }
        if (defl > 0.0 && piv <= defl) {
            for (int r = c + tid; r < k; r += nt) P[pk(r, c, k)] = 0.0;
        } else {
            const double inv = 1.0 / sqrt(piv);
            for (int r = c + tid; r < k; r += nt) P[pk(r, c, k)] = (r == c) ? sqrt(piv) : part[r] * inv;
        }
        __syncthreads();
    }
    return true;
}

__global__ __launch_bounds__(kSmallThreads) void k_chol_small(const SmallDesc *__restrict__ descs,
                                                               int mode, DevParams *params) {
    __shared__ double lds[kCholLds];
    __shared__ double part[2 * kMaxSketch];
    __shared__ double red[kSmallThreads / 64];
    __shared__ int s_fail;
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    if (k <= 0) return;
    const int tid = threadIdx.x;
    const bool packed = (k > kLdsK) && (k <= kPackK);
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
    if (packed) {
        for (int q = 0; q < k; ++q)
            for (int r = q + tid; r < k; r += blockDim.x)
                lds[pk(r, q, k)] = d.A[r + (int64_t)q * d.lda] + ((r == q) ? shift : 0.0);
    } else {
        for (int e = tid; e < k * k; e += blockDim.x) {
            const int r = e % k, q = e / k;
            if (r >= q) W[r + q * ldw] = d.A[r + (int64_t)q * d.lda] + ((r == q) ? shift : 0.0);
        }
    }
    __syncthreads();
    bool ok;
    if (packed) {
        ok = chol_packed(lds, k, defl, part, &s_fail);
        if (ok) {
            for (int e = tid; e < k * k; e += blockDim.x) {
                const int r = e % k, q = e / k;
                d.R[r + (int64_t)q * d.ldr] = (r <= q) ? lds[pk(q, r, k)] : 0.0;
            }
            return;
        }
    } else if (k <= kLdsK) {
        ok = chol_inplace(W, ldw, k, defl, part, &s_fail);
    } else {
        __syncthreads();
        ok = chol_blocked_global(W, ldw, k, defl, lds, part, &s_fail);
    }
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
constexpr int kTrsmLds = 176;

// Forward substitution of one row y against upper-triangular R, CH columns
// at a time; the block R[0:c0+CH, c0:c0+CH] is staged in LDS by the whole
// work-group (one wave) so the inner loop reads it as a broadcast.
constexpr int kTrsmCh = 8;
__device__ void row_solve(double *yrow, int64_t stride, int k, const double *__restrict__ R, int64_t ldr,
                          double *Rb, bool valid) {
    constexpr int CH = kTrsmCh;
    const int t = threadIdx.x;
    for (int c0 = 0; c0 < k; c0 += CH) {
        const int cw = (k - c0 < CH) ? (k - c0) : CH;
        const int rows = c0 + cw;
        __syncthreads();
        for (int e = t; e < rows * CH; e += blockDim.x) {
            const int q = e / CH, j = e - q * CH;
            Rb[e] = (j < cw) ? R[q + (int64_t)(c0 + j) * ldr] : 0.0;
        }
        __syncthreads();
        if (!valid) continue;
        double acc[CH];
#pragma unroll
        for (int j = 0; j < CH; ++j) acc[j] = (j < cw) ? yrow[(c0 + j) * stride] : 0.0;
        for (int q = 0; q < c0; ++q) {
            const double v = yrow[q * stride];
            const double *rq = Rb + q * CH;
#pragma unroll
            for (int j = 0; j < CH; ++j) acc[j] -= v * rq[j];
        }
#pragma unroll
        for (int j = 0; j < CH; ++j) {
            if (j < cw) {
                double a = acc[j];
#pragma unroll
                for (int jp = 0; jp < CH; ++jp)
                    if (jp < j) a -= acc[jp] * Rb[(c0 + jp) * CH + j];
                const double rd = Rb[(c0 + j) * CH + j];
                acc[j] = (rd != 0.0) ? a / rd : 0.0;  // zero diagonal: dead direction
            }
        }
#pragma unroll
        for (int j = 0; j < CH; ++j)
            if (j < cw) yrow[(c0 + j) * stride] = acc[j];
    }
}

__global__ __launch_bounds__(64) void k_trsm_rows(const SmallDesc *__restrict__ descs) {
    __shared__ double Yt[kTrsmLds * 64];
    __shared__ double Rb[kMaxSketch * kTrsmCh];
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
        row_solve(Yt + t, 64, k, d.R, d.ldr, Rb, true);
        if (valid)
            for (int c = 0; c < k; ++c) d.Y[row + c * ldy] = Yt[c * 64 + t];
    } else {
        row_solve(d.Y + (valid ? row : 0), ldy, k, d.R, d.ldr, Rb, valid);
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

// --------------------------------------------- truncated pivoted QR --

// Householder QR with column pivoting of A (k x k), stopped at the first step
// c where the Frobenius norm of the trailing block is <= tol:
//     A Pi = Q [R11 R12; 0 R22],  ||R22||_F <= tol,
// so A ~ Q1 B with Q1 = Q[:, :r] (k x r, orthonormal) and B = [R11 R12] Pi^T
// (r x k), spectral error <= tol.  Outputs: X = Q1 (ldx), Y = B^T (k x r, ldy),
// rank = {r, r}, flag = 0 (a rank above rank_cap sets TLR_RANK_OVERFLOW and
// is capped).  The working copy is row-major (element (i, j) at i*ld + j) so
// that the thread owning column j and its neighbours touch consecutive words.
template <int THREADS>
__device__ void qrcp_trunc(double *M, int ld, int k, double tol2, double *cn, double *beta, int *perm,
                           double *red, int *ired, int *s_r) {
    const int tid = threadIdx.x;
    for (int j = tid; j < k; j += THREADS) {
        double s2 = 0.0;
        for (int i = 0; i < k; ++i) s2 += M[i * ld + j] * M[i * ld + j];
        cn[j] = s2;
        perm[j] = j;
    }
    __syncthreads();
    int c = 0;
    for (; c < k; ++c) {
        // trailing Frobenius^2 and pivot (largest norm, smallest index on ties)
        double rem = 0.0, best = -1.0;
        int bj = c;
        for (int j = c + tid; j < k; j += THREADS) {
            rem += cn[j];
            if (cn[j] > best) { best = cn[j]; bj = j; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            rem += __shfl_xor(rem, off, 64);
            const double ob = __shfl_xor(best, off, 64);
            const int oj = __shfl_xor(bj, off, 64);
            if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
        }
        const int lane = tid & 63, wave = tid >> 6;
        if (lane == 0) { red[wave] = rem; red[8 + wave] = best; ired[wave] = bj; }
        __syncthreads();
        rem = 0.0; best = -1.0; bj = c;
        for (int w = 0; w < THREADS / 64; ++w) {
            rem += red[w];
            if (red[8 + w] > best || (red[8 + w] == best && ired[w] < bj)) { best = red[8 + w]; bj = ired[w]; }
        }
        if (rem <= tol2) break;
        __syncthreads();
        if (bj != c) {  // swap columns c and bj (all rows), norms and permutation
            for (int i = tid; i < k; i += THREADS) {
                const double t = M[i * ld + c];
                M[i * ld + c] = M[i * ld + bj];
                M[i * ld + bj] = t;
            }
            if (tid == 0) {
                const double t = cn[c]; cn[c] = cn[bj]; cn[bj] = t;
                const int q = perm[c]; perm[c] = perm[bj]; perm[bj] = q;
            }
        }
        __syncthreads();
        // Householder vector of M[c:, c]: v = x - alpha e1, beta = 2 / v^T v
        double x2 = 0.0;
        for (int i = c + 1 + tid; i < k; i += THREADS) x2 += M[i * ld + c] * M[i * ld + c];
        for (int off = 32; off > 0; off >>= 1) x2 += __shfl_xor(x2, off, 64);
        if (lane == 0) red[16 + wave] = x2;
        __syncthreads();
        x2 = 0.0;
        for (int w = 0; w < THREADS / 64; ++w) x2 += red[16 + w];
        const double x0 = M[c * ld + c];
        const double nrm = sqrt(x0 * x0 + x2);
        const double alpha = (x0 > 0.0) ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double vtv = v0 * v0 + x2;
        const double bta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
        __syncthreads();
        if (tid == 0) {
            M[c * ld + c] = v0;  // v stored in column c rows c..k-1 until the end
            beta[c] = bta;
        }
        __syncthreads();
        // apply to the trailing columns and refresh their norms
        for (int j = c + 1 + tid; j < k; j += THREADS) {
            double w = 0.0;
            for (int i = c; i < k; ++i) w += M[i * ld + c] * M[i * ld + j];
            w *= bta;
            double s2 = 0.0;
            for (int i = c; i < k; ++i) {
                const double nv = M[i * ld + j] - w * M[i * ld + c];
                M[i * ld + j] = nv;
                if (i > c) s2 += nv * nv;
            }
            cn[j] = s2;
        }
        __syncthreads();
        if (tid == 0) red[24] = alpha;
        __syncthreads();
        // keep alpha (the R diagonal) aside: column c below the diagonal holds v
        if (tid == 0) cn[c] = red[24];
        __syncthreads();
    }
    if (tid == 0) *s_r = c;
    __syncthreads();
}

// Register-resident variant for kJacK < k <= S*KH, 256*S threads: column j
// is held in registers by threads j + 256 h, h = 0..S-1, each owning rows
// [h KH, (h+1) KH); loops are fully unrolled with the row range as a predicate
// so the arrays stay in VGPRs.  Partial dot products / norms of the S parts
// meet in LDS.  Same arithmetic as qrcp_trunc.  vstore: k x k global scratch
// holding the reflectors.
template <int KH, int S>
__device__ void qrcp_reg(const SmallDesc &d, int k, double tol2, int min_tail, int k_full, int rank_cap,
                         DevParams *params, double *vstore) {
    __shared__ double sv[S * KH];
    __shared__ double part[S][256], part2[S][256];
    __shared__ double cn[256];
    __shared__ double beta[S * KH];
    __shared__ double alph[S * KH];
    __shared__ int perm[256];
    __shared__ double red[24];
    __shared__ int ired[8];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = tid & 255, h = tid >> 8, row0 = h * KH;
    const bool own = j < k;
    double col[KH];
#pragma unroll
    for (int ii = 0; ii < KH; ++ii)
        col[ii] = (own && row0 + ii < k) ? d.A[(row0 + ii) + (int64_t)j * d.lda] : 0.0;
    {
        double s2 = 0.0;
#pragma unroll
        for (int ii = 0; ii < KH; ++ii) s2 += col[ii] * col[ii];
        part[h][j] = s2;
    }
    __syncthreads();
    if (h == 0) {
        double t = 0.0;
        for (int q = 0; q < S; ++q) t += part[q][j];
        cn[j] = own ? t : -1.0;
        perm[j] = j;
    }
    __syncthreads();
    int c = 0;
    for (; c < k; ++c) {
        if (h == 0) {
            const bool act = own && j >= c;
            double rem = act ? cn[j] : 0.0, best = act ? cn[j] : -1.0;
            int bj = act ? j : k;
            for (int off = 32; off > 0; off >>= 1) {
                rem += __shfl_xor(rem, off, 64);
                const double ob = __shfl_xor(best, off, 64);
                const int oj = __shfl_xor(bj, off, 64);
                if (ob > best || (ob == best && oj < bj)) { best = ob; bj = oj; }
            }
            if (lane == 0) { red[wave] = rem; red[8 + wave] = best; ired[wave] = bj; }
        }
        __syncthreads();
        double rem = 0.0, best = -1.0;
        int bj = k;
        for (int w = 0; w < 4; ++w) {
            rem += red[w];
            if (red[8 + w] > best || (red[8 + w] == best && ired[w] < bj)) { best = red[8 + w]; bj = ired[w]; }
        }
        if (rem <= tol2) break;
        __syncthreads();
        if (bj != c) {  // swap columns c and bj through LDS, both halves
            if (j == bj) {
#pragma unroll
                for (int ii = 0; ii < KH; ++ii) sv[row0 + ii] = col[ii];
            }
            __syncthreads();
            if (j == c) {
#pragma unroll
                for (int ii = 0; ii < KH; ++ii) {
                    const double t = col[ii];
                    col[ii] = sv[row0 + ii];
                    sv[row0 + ii] = t;
                }
            }
            __syncthreads();
            if (j == bj) {
#pragma unroll
                for (int ii = 0; ii < KH; ++ii) col[ii] = sv[row0 + ii];
            }
            if (tid == 0) {
                const double t = cn[c]; cn[c] = cn[bj]; cn[bj] = t;
                const int q = perm[c]; perm[c] = perm[bj]; perm[bj] = q;
            }
            __syncthreads();
        }
        // Householder vector of column c: partial sums of both halves
        if (j == c) {
            double x2 = 0.0, x0 = 0.0;
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) {
                const int i = row0 + ii;
                if (i == c) x0 = col[ii];
                if (i > c) x2 += col[ii] * col[ii];
            }
            part[h][0] = x2;
            part2[h][0] = x0;
        }
        __syncthreads();
        if (tid == 0) {
            double x2 = 0.0, x0 = 0.0;
            for (int q = 0; q < S; ++q) {
                x2 += part[q][0];
                x0 += part2[q][0];
            }
            const double nrm = sqrt(x0 * x0 + x2);
            const double alpha = (x0 > 0.0) ? -nrm : nrm;
            const double v0 = x0 - alpha;
            const double vtv = v0 * v0 + x2;
            beta[c] = (vtv > 0.0) ? 2.0 / vtv : 0.0;
            alph[c] = alpha;
            red[16] = v0;
        }
        __syncthreads();
        if (j == c) {
            const double v0 = red[16];
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) {
                const int i = row0 + ii;
                const double vi = (i < c) ? 0.0 : (i == c ? v0 : col[ii]);
                sv[i] = vi;
                if (i < k) vstore[i + (int64_t)c * k] = vi;
            }
        }
        __syncthreads();
        const bool upd = own && j > c;
        if (upd) {
            double w = 0.0;
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) w += sv[row0 + ii] * col[ii];
            part[h][j] = w;
        }
        __syncthreads();
        if (upd) {
            double w = 0.0;
            for (int q = 0; q < S; ++q) w += part[q][j];
            w *= beta[c];
            double s2 = 0.0;
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) {
                col[ii] -= w * sv[row0 + ii];
                if (row0 + ii > c) s2 += col[ii] * col[ii];
            }
            part2[h][j] = s2;
        }
        __syncthreads();
        if (h == 0 && upd) {
            double t = 0.0;
            for (int q = 0; q < S; ++q) t += part2[q][j];
            cn[j] = t;
        }
        __syncthreads();
    }
    const int rr = c;
    const int insufficient = (k - rr < min_tail) && (k < (d.k_full < k_full ? d.k_full : k_full));
    int r = insufficient ? 0 : rr;
    if (!insufficient && r > rank_cap) {
        if (tid == 0) set_status(params, TLR_RANK_OVERFLOW, d.tile_i, d.tile_j);
        r = rank_cap;
    }
    // B^T: column j of R (rows < r) goes to Y[perm[j], :]
    if (own) {
#pragma unroll
        for (int ii = 0; ii < KH; ++ii) {
            const int i = row0 + ii;
            if (i < r) {
                const double v = (i < j) ? col[ii] : (i == j ? alph[i] : 0.0);
                d.Y[perm[j] + (int64_t)i * d.ldy] = v;
            }
        }
    }
    // Q1 = H_0 ... H_{r-1} [I_r; 0]: column q in the registers of threads q, q+256
    double qc[KH];
#pragma unroll
    for (int ii = 0; ii < KH; ++ii) qc[ii] = (row0 + ii == j) ? 1.0 : 0.0;
    for (int cc = r - 1; cc >= 0; --cc) {
        __syncthreads();
        for (int i = tid; i < S * KH; i += 256 * S) sv[i] = (i < k) ? vstore[i + (int64_t)cc * k] : 0.0;
        __syncthreads();
        if (j < r) {
            double w = 0.0;
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) w += sv[row0 + ii] * qc[ii];
            part[h][j] = w;
        }
        __syncthreads();
        if (j < r) {
            double w = 0.0;
            for (int q = 0; q < S; ++q) w += part[q][j];
            w *= beta[cc];
#pragma unroll
            for (int ii = 0; ii < KH; ++ii) qc[ii] -= w * sv[row0 + ii];
        }
    }
    if (j < r) {
#pragma unroll
        for (int ii = 0; ii < KH; ++ii)
            if (row0 + ii < k) d.X[(row0 + ii) + (int64_t)j * d.ldx] = qc[ii];
    }
    if (tid == 0) {
        d.rank[0] = r;
        d.rank[1] = rr;
        *d.flag = insufficient;
    }
}

__global__ __launch_bounds__(1024) void k_qrcp_reg(const SmallDesc *__restrict__ descs, double tol, int min_tail,
                                                    int k_full, int rank_cap, DevParams *params) {
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    if (k <= kJacK || k > kRegK) return;  // handled by k_qrcp_trunc
    qrcp_reg<kRegK / 4, 4>(d, k, tol * tol, min_tail, k_full, rank_cap, params, d.R);
}

__global__ __launch_bounds__(256) void k_qrcp_trunc(const SmallDesc *__restrict__ descs, double tol, int min_tail,
                                                     int k_full, int rank_cap, DevParams *params) {
    __shared__ double lds[kJacK * (kJacK + 1)];
    __shared__ double cn[kMaxSketch];
    __shared__ double beta[kMaxSketch];
    __shared__ int perm[kMaxSketch];
    __shared__ double red[32];
    __shared__ int ired[8];
    __shared__ int s_r;
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    const int tid = threadIdx.x;
    if (k <= 0 || k > kMaxSketch) {
        if (tid == 0) {
            d.rank[0] = d.rank[1] = 0;
            *d.flag = 0;
            if (k > kMaxSketch) set_status(params, TLR_RANK_OVERFLOW, d.tile_i, d.tile_j);
        }
        return;
    }
    if (k > kJacK && k <= kRegK) return;  // k_qrcp_reg
    double *M = (k <= kJacK) ? lds : d.R;  // row-major working copy
    const int ldm = (k <= kJacK) ? k + 1 : k;
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, j = e - (e / k) * k;
        M[i * ldm + j] = d.A[i + (int64_t)j * d.lda];
    }
    __syncthreads();
    qrcp_trunc<256>(M, ldm, k, tol * tol, cn, beta, perm, red, ired, &s_r);
    // a rank within min_tail of the sample width means the sample was too
    // narrow: keep the previous factors (rank 0 written) and let the host retry
    const int insufficient = (k - s_r < min_tail) && (k < (d.k_full < k_full ? d.k_full : k_full));
    int r = insufficient ? 0 : s_r;
    if (!insufficient && r > rank_cap) {
        if (tid == 0) set_status(params, TLR_RANK_OVERFLOW, d.tile_i, d.tile_j);
        r = rank_cap;
    }
    // Y = B^T (k x r): B[c][perm[j]] = R[c][j] for j >= c (R[c][c] = alpha_c, kept in cn[c])
    for (int e = tid; e < k * r; e += 256) {
        const int c = e / k, j = e - c * k;  // row c of B, column j (pivoted order)
        double v;
        if (j < c) v = 0.0;
        else if (j == c) v = cn[c];
        else v = M[c * ldm + j];
        d.Y[perm[j] + (int64_t)c * d.ldy] = v;
    }
    // X = Q1 = H_0 ... H_{r-1} [I_r; 0], backward accumulation, column q by thread
    for (int q = tid; q < r; q += 256) {
        double *xq = d.X + (int64_t)q * d.ldx;
        for (int i = 0; i < k; ++i) xq[i] = (i == q) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int c = r - 1; c >= 0; --c) {
        const double bta = beta[c];
        for (int q = tid; q < r; q += 256) {
            double *xq = d.X + (int64_t)q * d.ldx;
            double w = 0.0;
            for (int i = c; i < k; ++i) w += M[i * ldm + c] * xq[i];
            w *= bta;
            for (int i = c; i < k; ++i) xq[i] -= w * M[i * ldm + c];
        }
        __syncthreads();
    }
    if (tid == 0) {
        d.rank[0] = r;
        d.rank[1] = s_r;
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
                      hipStream_t s, const SmallDesc *h_descs) {
    (void)max_k;
    if (count <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_chol_small");
    double flops = 0.0, bytes = 0.0;
    if (h_descs && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const double k = h_descs[t].k;
            flops += k * k * k / 3.0;
            bytes += 8.0 * k * (k + 1.0);  // lower triangle in, upper factor out
        }
    KTimer kt(cls, s, flops, bytes, h_descs != nullptr);
    hipLaunchKernelGGL(k_chol_small, dim3(count), dim3(kSmallThreads), 0, s, d_descs, mode, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status trsm_rows(const SmallDesc *d_descs, int count, int max_m, int max_k, hipStream_t s,
                     const SmallDesc *h_descs) {
    (void)max_k;
    if (count <= 0 || max_m <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_trsm_rows");
    double flops = 0.0, bytes = 0.0;
    if (h_descs && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const double k = h_descs[t].k, m = h_descs[t].m;
            flops += m * k * k;
            bytes += 8.0 * (2.0 * m * k + k * (k + 1.0) / 2.0);
        }
    KTimer kt(cls, s, flops, bytes, h_descs != nullptr);
    hipLaunchKernelGGL(k_trsm_rows, dim3((unsigned)cdiv(max_m, 64), count), dim3(64), 0, s, d_descs);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status jacobi_svd(const SmallDesc *d_descs, int count, int max_k, double tol, int min_tail,
                      int k_full, int rank_cap, DevParams *params, hipStream_t s) {
    (void)max_k;
    if (count <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_jacobi_svd");
    KTimer kt(cls, s, 0.0, 0.0, false);  // iterative: no fixed operation count
    hipLaunchKernelGGL(k_jacobi_svd, dim3(count), dim3(kSmallThreads), 0, s, d_descs, tol, min_tail,
                       k_full, rank_cap, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status qrcp_trunc(const SmallDesc *d_descs, int count, int max_k, double tol, int min_tail, int k_full,
                      int rank_cap, DevParams *params, hipStream_t s) {
    if (count <= 0) return TLR_OK;
    static const int cls_t = ktimer_class("k_qrcp_trunc"), cls_r = ktimer_class("k_qrcp_reg");
    {
        // the stopping step (the rank) is decided on the device
        KTimer kt(cls_t, s, 0.0, 0.0, false);
        hipLaunchKernelGGL(k_qrcp_trunc, dim3(count), dim3(256), 0, s, d_descs, tol, min_tail, k_full, rank_cap,
                           params);
    }
    if (max_k > kJacK) {
        KTimer kt(cls_r, s, 0.0, 0.0, false);
        hipLaunchKernelGGL(k_qrcp_reg, dim3(count), dim3(1024), 0, s, d_descs, tol, min_tail, k_full, rank_cap,
                           params);
    }
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
