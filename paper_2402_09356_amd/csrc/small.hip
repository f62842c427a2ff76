// Batched small dense kernels, one work-group per problem:
//  * one-sided (Hestenes) Jacobi SVD of a k x k matrix,
//  * truncated pivoted QR of a k x k matrix,
// plus the block triangular solve of the panel factors against a diagonal tile.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "ktimer.h"
#include "lanes.h"

namespace tlr {
namespace {

constexpr int kSmallThreads = 256;
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
            rank_overflow(params, d.tile_i, d.tile_j);
            write = rank_cap;
        }
        if (insufficient) write = 0;  // keep the previous factors; the host retries wider
        d.rank[0] = write;  // rank used to form the new factors
        d.rank[1] = r;      // numerical rank seen by this sample
        *d.flag = insufficient;
    }
}

// --------------------------------------------- truncated pivoted QR --

// Squared stopping threshold of the truncation: tol^2, or with float32
// factors (floor_rel > 0) max(tol, floor_rel (||A||_F + noise))^2, where
// ||A||_F^2 = total2 is the whole matrix's squared Frobenius norm and noise
// the rounding-noise norm of the operator the sketch was taken of: directions
// below that level are float32 rounding, not rank.
__device__ inline double trunc_thr2(const DevParams *params, const double *noise, double total2, double tol2) {
    const double rel = params->floor_rel;
    if (!(rel > 0.0)) return tol2;
    const double f = rel * (sqrt(total2) + (noise ? *noise : 0.0));
    return fmax(tol2, f * f);
}

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
                           double *red, int *ired, int *s_r, const DevParams *params, const double *noise) {
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
        {
            // the waves' entries read at once, then combined in registers
            double rv[THREADS / 64], bv[THREADS / 64];
            int iv[THREADS / 64];
#pragma unroll
            for (int w = 0; w < THREADS / 64; ++w) {
                rv[w] = red[w];
                bv[w] = red[8 + w];
                iv[w] = ired[w];
            }
#pragma unroll
            for (int w = 0; w < THREADS / 64; ++w) {
                rem += rv[w];
                const bool take = bv[w] > best || (bv[w] == best && iv[w] < bj);
                best = take ? bv[w] : best;
                bj = take ? iv[w] : bj;
            }
        }
        if (c == 0) tol2 = trunc_thr2(params, noise, rem, tol2);
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
        // apply to the trailing columns and refresh their norms; eight rows
        // at a time so that the loads of a batch are in flight together
        for (int j = c + 1 + tid; j < k; j += THREADS) {
            double w8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int i = c;
            for (; i + 8 <= k; i += 8) {
                double vv[8], xx[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    vv[u] = M[(i + u) * ld + c];
                    xx[u] = M[(i + u) * ld + j];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) w8[u] += vv[u] * xx[u];
            }
            for (; i < k; ++i) w8[0] += M[i * ld + c] * M[i * ld + j];
            double w = ((w8[0] + w8[1]) + (w8[2] + w8[3])) + ((w8[4] + w8[5]) + (w8[6] + w8[7]));
            w *= bta;
            const double nc = M[c * ld + j] - w * M[c * ld + c];
            M[c * ld + j] = nc;
            double s8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            i = c + 1;
            for (; i + 8 <= k; i += 8) {
                double vv[8], xx[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    vv[u] = M[(i + u) * ld + c];
                    xx[u] = M[(i + u) * ld + j];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const double nv = xx[u] - w * vv[u];
                    M[(i + u) * ld + j] = nv;
                    s8[u] += nv * nv;
                }
            }
            for (; i < k; ++i) {
                const double nv = M[i * ld + j] - w * M[i * ld + c];
                M[i * ld + j] = nv;
                s8[0] += nv * nv;
            }
            cn[j] = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
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

// Register-resident variant for k <= 16 RPS and k <= 4 NW CPG (NW waves).
// The matrix is spread over 4 NW column groups of 16 lanes (a quarter-wave):
// group g owns columns g + 4 NW cc (cc < CPG), its lane s the rows s + 16 rr
// (rr < RPS), so a column's reductions are four DPP steps inside its group.
// Columns are never swapped: the pivot of step c is frozen in place (rows < c
// hold its column of R, row c the diagonal alpha_c, rows below c its
// Householder vector, whose first entry is kept aside).  Each step the owner
// group puts the pivot column in LDS and every group forms the reflector
// itself; the reflectors go to V (k x k scratch, column c) once, after the
// last step.  Same arithmetic as
// qrcp_trunc (pivot = largest remaining norm, smallest index on ties; stop
// when the remaining Frobenius norm is <= tol), so Y = B^T comes straight from
// the registers and Q1 is accumulated in registers from V.  The column norms
// stay in registers too: each step's pivot search reduces them within the
// wave and across waves through LDS, and a step needs two barriers.
template <int NW, int CPG, int RPS>
__global__ __launch_bounds__(NW * 64) void k_qrcp_regs(const SmallDesc *__restrict__ descs, double tol,
                                                        int min_tail, int k_full, int rank_cap, DevParams *params,
                                                        int kmin) {
    constexpr int G = 4 * NW, KC = G * CPG, KR = 16 * RPS, NT = NW * 64;
    constexpr int kNever = 1 << 30;
    __shared__ int pst[KC];  // step at which the column was pivoted (kNever: not yet)
    __shared__ double vsh[KR];
    __shared__ double bet[KR];
    __shared__ double v0s[KR];  // first entry of each step's Householder vector
    __shared__ double redv[2][2 * NW];  // per wave: trailing norm, best norm; by step parity
    __shared__ int redi[2][NW];
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    if (k <= 0 && kmin <= 1) {
        if (threadIdx.x == 0) {
            d.rank[0] = d.rank[1] = 0;
            *d.flag = 0;
        }
        return;
    }
    if (k < kmin || k > KC || k > KR) return;  // another kernel's range
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int grp = wave * 4 + (lane >> 4), sl = lane & 15;
    double tol2 = tol * tol;
    double *__restrict__ V = d.R;
    double a[CPG][RPS];
    // per column of the group: squared norm of its rows below the current
    // step (the same in all 16 lanes), and whether it is still unpivoted
    double cnr[CPG];
    bool act[CPG];
#pragma unroll
    for (int cc = 0; cc < CPG; ++cc) {
        const int p = grp + G * cc;
        double n2 = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) {
            const int i = sl + 16 * rr;
            a[cc][rr] = (p < k && i < k) ? d.A[i + (int64_t)p * d.lda] : 0.0;
            n2 += a[cc][rr] * a[cc][rr];
        }
        cnr[cc] = red16(n2);
        act[cc] = p < k;
    }
    for (int t = tid; t < KC; t += NT) pst[t] = kNever;
    __syncthreads();
    int c = 0;
    for (; c < k; ++c) {
        const int par = c & 1;
        // the wave's share of the pivot search, from the norms in registers:
        // its groups' columns, then its four groups (lanes 0, 16, 32, 48)
        double rem = 0.0, best = -1.0;
        int bj = k;
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) {
            const int p = grp + G * cc;
            if (act[cc]) {
                rem += cnr[cc];
                if (cnr[cc] > best || (cnr[cc] == best && p < bj)) {
                    best = cnr[cc];
                    bj = p;
                }
            }
        }
        {
            double rs[4], bs[4];
            int js[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                rs[q] = readlane_d(rem, 16 * q);
                bs[q] = readlane_d(best, 16 * q);
                js[q] = __builtin_amdgcn_readlane(bj, 16 * q);
            }
            rem = (rs[0] + rs[1]) + (rs[2] + rs[3]);
            best = bs[0];
            bj = js[0];
#pragma unroll
            for (int q = 1; q < 4; ++q)
                if (bs[q] > best || (bs[q] == best && js[q] < bj)) {
                    best = bs[q];
                    bj = js[q];
                }
        }
        if (lane == 0) {
            redv[par][wave] = rem;
            redv[par][NW + wave] = best;
            redi[par][wave] = bj;
        }
        __syncthreads();
        {
            // all the waves' entries read at once, then combined in registers
            // (a read inside the comparison chain would put one LDS round
            // trip per wave on the step's critical path)
            double rv[NW], bv[NW];
            int iv[NW];
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                rv[w] = redv[par][w];
                bv[w] = redv[par][NW + w];
                iv[w] = redi[par][w];
            }
            rem = 0.0;
            best = -1.0;
            bj = k;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                rem += rv[w];
                const bool take = bv[w] > best || (bv[w] == best && iv[w] < bj);
                best = take ? bv[w] : best;
                bj = take ? iv[w] : bj;
            }
        }
        // every lane holds the same values: in scalar registers the branches
        // on them below are scalar too (the owner group's column loops then
        // run one column's code, not six behind exec masks)
        bj = __builtin_amdgcn_readfirstlane(bj);
        rem = readlane_d(rem, 0);
        if (c == 0) tol2 = trunc_thr2(params, d.noise, rem, tol2);
        if (rem <= tol2) break;
        // the pivot column (rows c .. k-1) into LDS, by the group that owns it
        if (grp == bj % G) {
            const int oc = bj / G;
#pragma unroll
            for (int cc = 0; cc < CPG; ++cc)
                if (cc == oc) {
                    act[cc] = false;
#pragma unroll
                    for (int rr = 0; rr < RPS; ++rr) {
                        const int i = sl + 16 * rr;
                        vsh[i] = (i < c || i >= k) ? 0.0 : a[cc][rr];
                    }
                }
            if (sl == 0) pst[bj] = c;
        }
        __syncthreads();
        // every group forms the Householder vector v = x - alpha e_c of the
        // shared column, each with the sums its owner would form (the same
        // terms in the same order), so every lane holds the same values
        double vr[RPS];
        double x2 = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) {
            vr[rr] = vsh[sl + 16 * rr];
            if (sl + 16 * rr > c) x2 += vr[rr] * vr[rr];
        }
        x2 = red16(x2);
        const double x0 = vsh[c];
        const double nrm = sqrt(x0 * x0 + x2);
        const double alpha = (x0 > 0.0) ? -nrm : nrm;
        const double v0 = x0 - alpha;
        const double vtv = v0 * v0 + x2;
        const double bta = (vtv > 0.0) ? 2.0 / vtv : 0.0;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr)
            if (sl + 16 * rr == c) vr[rr] = v0;
        if (grp == bj % G) {  // R's diagonal entry replaces x_c in the frozen column
            const int oc = bj / G;
#pragma unroll
            for (int cc = 0; cc < CPG; ++cc)
                if (cc == oc) {
#pragma unroll
                    for (int rr = 0; rr < RPS; ++rr)
                        if (sl + 16 * rr == c) a[cc][rr] = alpha;
                }
        }
        if (tid == 0) {
            bet[c] = bta;
            v0s[c] = v0;
        }
        // row blocks wholly above row c are finished: the reflector is zero
        // there, so they are skipped (one uniform branch per block; the terms
        // left out are exact zeros, so every sum keeps its bits)
        const int rb0 = c >> 4;
        double w[CPG];
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) w[cc] = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) {
            if (rr < rb0) continue;
#pragma unroll
            for (int cc = 0; cc < CPG; ++cc) w[cc] += vr[rr] * a[cc][rr];
        }
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) w[cc] = red16(act[cc] ? w[cc] : 0.0) * bta;
        double n2[CPG];
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) n2[cc] = 0.0;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) {
            if (rr < rb0) continue;
            const int i = sl + 16 * rr;
            const bool below = i > c && i < k;
#pragma unroll
            for (int cc = 0; cc < CPG; ++cc) {
                a[cc][rr] -= w[cc] * vr[rr];
                if (below) n2[cc] += a[cc][rr] * a[cc][rr];
            }
        }
        // the new norms stay in registers; the next step's search needs no
        // barrier before it (it writes the other parity's slots, and vsh and
        // bet are rewritten only after its barrier)
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) cnr[cc] = red16(n2[cc]);
    }
    const int rr_rank = c;
    const int insufficient = (k - rr_rank < min_tail) && (k < (d.k_full < k_full ? d.k_full : k_full));
    int r = insufficient ? 0 : rr_rank;
    if (!insufficient && r > rank_cap) {
        if (tid == 0) rank_overflow(params, d.tile_i, d.tile_j);
        r = rank_cap;
    }
    // Y = B^T: B[i][p] = R entry for i <= pivot step of p (the diagonal sits
    // at the pivot step), 0 below
#pragma unroll
    for (int cc = 0; cc < CPG; ++cc) {
        const int p = grp + G * cc;
        if (p < k) {
            const int ps = pst[p];
#pragma unroll
            for (int rr = 0; rr < RPS; ++rr) {
                const int i = sl + 16 * rr;
                if (i < r) d.Y[p + (int64_t)i * d.ldy] = (i <= ps) ? a[cc][rr] : 0.0;
            }
        }
    }
    __syncthreads();  // v0s and pst of the last step visible to every wave
    // the reflectors into V: the column pivoted at step h holds v below row h
    // (frozen since), and v_h was kept aside
#pragma unroll
    for (int cc = 0; cc < CPG; ++cc) {
        const int p = grp + G * cc;
        const int h = (p < k) ? pst[p] : kNever;
        if (h < rr_rank) {
#pragma unroll
            for (int rr = 0; rr < RPS; ++rr) {
                const int i = sl + 16 * rr;
                if (i >= h && i < k) V[i + (int64_t)h * k] = (i == h) ? v0s[h] : a[cc][rr];
            }
        }
    }
    __syncthreads();  // reflectors in V visible to every wave
    // Q1 = H_0 ... H_{r-1} [I_r; 0]: column q held like matrix column q
#pragma unroll
    for (int cc = 0; cc < CPG; ++cc) {
        const int q = grp + G * cc;
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) a[cc][rr] = (sl + 16 * rr == q) ? 1.0 : 0.0;
    }
    // the reflectors go through LDS sixteen at a time, the next sixteen
    // loaded into registers while the current ones are applied
    constexpr int HC = 16, VL = HC * KR / NT;
    static_assert(VL * NT == HC * KR, "reflector chunk must split evenly over the threads");
    __shared__ double Vs[HC * KR];
    double vbuf[VL];
    auto vload = [&](int hc0) {
#pragma unroll
        for (int u = 0; u < VL; ++u) {
            const int e = tid + NT * u, hh = e / KR, i = e - hh * KR, h = hc0 - hh;
            vbuf[u] = (h >= 0 && i >= h && i < k) ? V[i + (int64_t)h * k] : 0.0;
        }
    };
    if (r > 0) vload(r - 1);
    for (int hc0 = r - 1; hc0 >= 0; hc0 -= HC) {
        __syncthreads();  // the previous chunk has been applied
#pragma unroll
        for (int u = 0; u < VL; ++u) Vs[tid + NT * u] = vbuf[u];
        __syncthreads();
        if (hc0 - HC >= 0) vload(hc0 - HC);
        const int hlo = hc0 - HC + 1 > 0 ? hc0 - HC + 1 : 0;
    for (int h = hc0; h >= hlo; --h) {
        double vr[RPS];
#pragma unroll
        for (int rr = 0; rr < RPS; ++rr) vr[rr] = Vs[(hc0 - h) * KR + sl + 16 * rr];
        const double bt = bet[h];
#pragma unroll
        for (int cc = 0; cc < CPG; ++cc) {
            const int q = grp + G * cc;
            double t = 0.0;
#pragma unroll
            for (int rr = 0; rr < RPS; ++rr) t += vr[rr] * a[cc][rr];
            t = red16(t) * bt;
            if (q < r && q >= h) {
#pragma unroll
                for (int rr = 0; rr < RPS; ++rr) a[cc][rr] -= t * vr[rr];
            }
        }
    }
    }
#pragma unroll
    for (int cc = 0; cc < CPG; ++cc) {
        const int q = grp + G * cc;
        if (q < r) {
#pragma unroll
            for (int rr = 0; rr < RPS; ++rr) {
                const int i = sl + 16 * rr;
                if (i < k) d.X[i + (int64_t)q * d.ldx] = a[cc][rr];
            }
        }
    }
    if (tid == 0) {
        d.rank[0] = r;
        d.rank[1] = rr_rank;
        *d.flag = insufficient;
    }
}

constexpr int kQrSmallK = 64;   // k_qrcp_regs<4, 4, 4>
constexpr int kQrMidK = 192;    // k_qrcp_regs<8, 6, 12>

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
    if (k <= kQrMidK) return;  // k_qrcp_regs
    double *M = (k <= kJacK) ? lds : d.R;  // row-major working copy
    const int ldm = (k <= kJacK) ? k + 1 : k;
    for (int e = tid; e < k * k; e += 256) {
        const int i = e / k, j = e - (e / k) * k;
        M[i * ldm + j] = d.A[i + (int64_t)j * d.lda];
    }
    __syncthreads();
    qrcp_trunc<256>(M, ldm, k, tol * tol, cn, beta, perm, red, ired, &s_r, params, d.noise);
    // a rank within min_tail of the sample width means the sample was too
    // narrow: keep the previous factors (rank 0 written) and let the host retry
    const int insufficient = (k - s_r < min_tail) && (k < (d.k_full < k_full ? d.k_full : k_full));
    int r = insufficient ? 0 : s_r;
    if (!insufficient && r > rank_cap) {
        if (tid == 0) rank_overflow(params, d.tile_i, d.tile_j);
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
            // eight rows at a time so that a batch's loads are in flight together
            double *xq = d.X + (int64_t)q * d.ldx;
            double w8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            int i = c;
            for (; i + 8 <= k; i += 8) {
                double vv[8], xx[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    vv[u] = M[(i + u) * ldm + c];
                    xx[u] = xq[i + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) w8[u] += vv[u] * xx[u];
            }
            for (; i < k; ++i) w8[0] += M[i * ldm + c] * xq[i];
            const double w = bta * (((w8[0] + w8[1]) + (w8[2] + w8[3])) + ((w8[4] + w8[5]) + (w8[6] + w8[7])));
            i = c;
            for (; i + 8 <= k; i += 8) {
                double vv[8], xx[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    vv[u] = M[(i + u) * ldm + c];
                    xx[u] = xq[i + u];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) xq[i + u] = xx[u] - w * vv[u];
            }
            for (; i < k; ++i) xq[i] -= w * M[i * ldm + c];
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

// Panels B_t[b0:b0+bs, :] <- L_bb^-1 B_t[b0:b0+bs, :], one work-group per
// (panel, chunk of 64 columns); L_bb is the diagonal block of L (ld nb).  The
// block of L and the 64 x 64 block of B go through LDS; wave w owns columns
// 16w..16w+15.  Four 16-row steps on the transposed block: the rows above
// are taken out with MFMA (solved rows x L rows), then the 16 x 16 diagonal
// block is solved along the lanes of each row of 16.  Rows past bs carry an
// identity diagonal (zero result).
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kTbP = 65;  // LDS pitch of both 64-row blocks

template <class T>
__global__ __launch_bounds__(256) void k_trsm_block(const double *__restrict__ L, int ldl, int b0, int bs,
                                                     const SmallDesc *__restrict__ descs) {
    __shared__ double Ls[64 * kTbP];  // Ls[r + c * kTbP] = L[b0 + r][b0 + c]
    __shared__ double Xs[64 * kTbP];  // Xs[r + c * kTbP]: row r, column c of the block of B
    const SmallDesc d = descs[blockIdx.y];
    T *__restrict__ Y = reinterpret_cast<T *>(d.Y);
    const int cols = d.k_dev ? *d.k_dev : d.k;
    const int c0 = blockIdx.x * 64;
    if (c0 >= cols) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    {
        // L (lower, identity past bs) and B, lane = row: sixteen loads each in flight
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = 4 * u + wave;  // columns wave, wave + 4, ...
            v[u] = (lane < bs && c < bs) ? (lane >= c ? L[(b0 + lane) + (int64_t)(b0 + c) * ldl] : 0.0)
                                         : ((lane == c) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) Ls[lane + (4 * u + wave) * kTbP] = v[u];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = 4 * u + wave, col = c0 + c;
            v[u] = (lane < bs && col < cols) ? (double)Y[(int64_t)col * d.ldy + b0 + lane] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) Xs[lane + (4 * u + wave) * kTbP] = v[u];
    }
    __syncthreads();
    const int wc = 16 * wave;  // this wave's first column
    // Each step works on the transpose of its 16 x 16 block (lane li holds
    // row r0 + li of the wave's columns wc + lg + 4 q), so the substitution
    // runs along the 16 lanes of a row: the solved entry of row j moves by
    // DPP and row li of L's diagonal block stays in registers.  A wave reads
    // and writes only its own columns, so the steps need no barrier.
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int r0 = 16 * s;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = Xs[(r0 + li) + (wc + lg + 4 * q) * kTbP];
        if (s > 0) {
            // rows r0..r0+15 -= L[r0.., 0:r0] X[0:r0, cols], as its transpose
            // X[0:r0, cols]^T L[r0.., 0:r0]^T
            v4d part = v4d{0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < r0; kk += 4) {
                const double av = Xs[(kk + lg) + (wc + li) * kTbP];
                const double bv = Ls[(r0 + li) + (kk + lg) * kTbP];
                part = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, part, 0, 0, 0);
            }
            acc -= part;
        }
        // diagonal block: lane li keeps row li unscaled until its own step
        // (the rows below leave it unchanged), then scales it
        double lj[16];  // L[r0 + li][r0 + j], strictly lower part
#pragma unroll
        for (int j = 0; j < 16; ++j) lj[j] = (j < li) ? Ls[(r0 + li) + (r0 + j) * kTbP] : 0.0;
        const double ivl = 1.0 / Ls[(r0 + li) + (r0 + li) * kTbP];
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            double mm[4], xc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) mm[q] = acc[q] * ivl;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) xc[q] = row_bcast_at(mm[q], j);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] -= xc[q] * lj[j];
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Xs[(r0 + li) + (wc + lg + 4 * q) * kTbP] = acc[q] * ivl;
        wave_sync();  // the solved rows are read across the wave's lanes next
    }
    __syncthreads();  // the write-back reads every wave's columns
    {
        // write back, lane = row
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int c = 4 * u + wave, col = c0 + c;
            if (lane < bs && col < cols) Y[(int64_t)col * d.ldy + b0 + lane] = (T)Xs[lane + c * kTbP];
        }
    }
}

}  // namespace

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
                      int rank_cap, DevParams *params, hipStream_t s, int min_k) {
    if (count <= 0) return TLR_OK;
    static const int cls_s = ktimer_class("k_qrcp_regs<4,4,4>"), cls_m = ktimer_class("k_qrcp_regs<8,6,12>"),
                     cls_t = ktimer_class("k_qrcp_trunc");
    // the stopping step (the rank) is decided on the device: no fixed count.
    // min_k: no descriptor is narrower (the kernels for narrower k are skipped)
    if (min_k <= kQrSmallK) {
        KTimer kt(cls_s, s, 0.0, 0.0, false);
        hipLaunchKernelGGL((k_qrcp_regs<4, 4, 4>), dim3(count), dim3(256), 0, s, d_descs, tol, min_tail, k_full,
                           rank_cap, params, 1);
    }
    if (max_k > kQrSmallK && min_k <= kQrMidK) {
        KTimer kt(cls_m, s, 0.0, 0.0, false);
        hipLaunchKernelGGL((k_qrcp_regs<8, 6, 12>), dim3(count), dim3(512), 0, s, d_descs, tol, min_tail, k_full,
                           rank_cap, params, kQrSmallK + 1);
    }
    if (max_k > kQrMidK) {
        KTimer kt(cls_t, s, 0.0, 0.0, false);
        hipLaunchKernelGGL(k_qrcp_trunc, dim3(count), dim3(256), 0, s, d_descs, tol, min_tail, k_full, rank_cap,
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

namespace {
__global__ void k_copy_batched(const CopyDesc *__restrict__ descs) {
    const CopyDesc d = descs[blockIdx.y];
    double *__restrict__ dst = static_cast<double *>(d.dst);
    if (d.conv == 1) {
        const float *__restrict__ src = static_cast<const float *>(d.src);
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.words;
             e += (int64_t)gridDim.x * blockDim.x)
            dst[e] = (double)src[e];
    } else if (d.conv == 2) {
        const float *__restrict__ src = static_cast<const float *>(d.src);
        float *__restrict__ fdst = static_cast<float *>(d.dst);
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.words;
             e += (int64_t)gridDim.x * blockDim.x)
            fdst[e] = src[e];
    } else {
        const double *__restrict__ src = static_cast<const double *>(d.src);
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < d.words;
             e += (int64_t)gridDim.x * blockDim.x)
            dst[e] = src[e];
    }
}

// ||V||_F of an nb x r float32 panel, one work-group a panel; partial sums
// combined in a fixed order (deterministic).
__global__ __launch_bounds__(256) void k_factor_norms(const NormDesc *__restrict__ descs, int nb) {
    __shared__ double part[256];
    const NormDesc d = descs[blockIdx.x];
    const int r = d.r_dev ? *d.r_dev : 0;
    const int64_t words = (int64_t)nb * (r > 0 ? r : 0);
    double acc = 0.0;
    for (int64_t e = threadIdx.x; e < words; e += 256) {
        const double v = (double)d.V[e];
        acc += v * v;
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *d.out = sqrt(part[0]);
}

// Rounding-noise norm of the Schur complement of tile (i, j), one thread a tile.
__global__ __launch_bounds__(64) void k_schur_noise(const NoiseDesc *__restrict__ descs, int count, int nt,
                                                    const double *__restrict__ nrm_s,
                                                    const double *__restrict__ nrm_l) {
    const int t = blockIdx.x * 64 + threadIdx.x;
    if (t >= count) return;
    const NoiseDesc d = descs[t];
    // the terms' rounding errors are independent: their norms add in quadrature
    const double s0 = nrm_s[(int64_t)d.i * nt + d.j];
    double acc = s0 * s0;
    for (int k = 0; k < d.j; ++k) {
        const double t = nrm_l[(int64_t)d.i * nt + k] * nrm_l[(int64_t)d.j * nt + k];
        acc += t * t;
    }
    *d.out = sqrt(acc);
}
}  // namespace

tlr_status factor_norms(const NormDesc *d_descs, int count, int nb, hipStream_t s) {
    if (count <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_factor_norms, dim3(count), dim3(256), 0, s, d_descs, nb);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status schur_noise(const NoiseDesc *d_descs, int count, int nt, const double *nrm_s, const double *nrm_l,
                       hipStream_t s) {
    if (count <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_schur_noise, dim3((unsigned)cdiv(count, 64)), dim3(64), 0, s, d_descs, count, nt, nrm_s,
                       nrm_l);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status copy_batched(const CopyDesc *d_descs, int count, int64_t max_words, hipStream_t s) {
    if (count <= 0 || max_words <= 0) return TLR_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(max_words, 256), 256);
    hipLaunchKernelGGL(k_copy_batched, dim3(gx, count), dim3(256), 0, s, d_descs);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

void trsm_left_lower_descs(const double *L, int nb, const SmallDesc *h_descs, int count, GemmDesc *h_gemm,
                           bool y32) {
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
            // the panel's rows b0.. and b0+bs.. in its own element type
            if (y32) {
                float *y = reinterpret_cast<float *>(pd.Y);
                o.B = y + b0;
                o.C = y + b0 + bs;
            } else {
                o.B = pd.Y + b0;
                o.C = pd.Y + b0 + bs;
            }
            o.ldb = pd.ldy;
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
}

tlr_status trsm_left_lower(const double *L, int nb, const SmallDesc *d_descs, const SmallDesc *h_descs,
                           int count, int max_cols, GemmDesc *d_gemm, GemmDesc *h_gemm, hipStream_t s, bool y32) {
    if (count <= 0 || max_cols <= 0) return TLR_OK;
    const int nblk = (int)cdiv(nb, 64);
    if (h_gemm) {  // else the caller has put the descriptors on the device
        trsm_left_lower_descs(L, nb, h_descs, count, h_gemm, y32);
        TLR_HIP(hipMemcpyAsync(d_gemm, h_gemm, sizeof(GemmDesc) * count * nblk, hipMemcpyHostToDevice, s));
    }
    static const int cls = ktimer_class("k_trsm_block");
    double cols_sum = 0.0;
    bool exact = h_descs != nullptr;
    if (exact)
        for (int t = 0; t < count; ++t) {
            if (h_descs[t].k_dev) exact = false;
            cols_sum += h_descs[t].k;
        }
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        {
            const double d = bs, wy = y32 ? 4.0 : 8.0;
            // bs^2 flops per right-hand side; the block of L once, each column read and written once
            KTimer kt(cls, s, d * d * cols_sum, 8.0 * d * (d + 1.0) / 2.0 + wy * 2.0 * d * cols_sum, exact);
            if (y32)
                hipLaunchKernelGGL((k_trsm_block<float>), dim3((unsigned)cdiv(max_cols, 64), count), dim3(256), 0, s,
                                   L, nb, b0, bs, d_descs);
            else
                hipLaunchKernelGGL((k_trsm_block<double>), dim3((unsigned)cdiv(max_cols, 64), count), dim3(256), 0, s,
                                   L, nb, b0, bs, d_descs);
        }
        if (rest > 0)
            TLR_TRY(gemm_batched(false, false, d_gemm + (int64_t)b * count, count, rest, max_cols, s, nullptr, false,
                                 y32 ? (kGemmB32 | kGemmC32) : 0));
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
