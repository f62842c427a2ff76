// The two halves of one CholeskyQR pass on the matrix cores:
//  * k_chol_small: Cholesky of a k x k Gram matrix (shifted CholeskyQR,
//    Fukaya, Kannan, Nakatsukasa, Zhang, Yamamoto, SIAM J. Sci. Comput. 2020;
//    deflation of null directions), right-looking over 16 x 16 tiles;
//  * k_trsm_rows: Y <- Y R^-1 for the m x k panel, 16 columns at a time
//    (the row block held in LDS; k_trsm_rows_wide for k above 192 and for
//    batches too large for one LDS-bound work-group per compute unit).
//
// Tiles.  The lower triangle is held as 16 x 16 tiles, tile (i, j), i >= j,
// at index i(i+1)/2 + j, each stored column-major with a column pitch of 17
// words (the pitch keeps both MFMA operand reads and accumulator writes free
// of bank conflicts).  Up to 11 tile rows (k <= 176) live in LDS, sized per
// launch; beyond that the tiles live in the job's k x k scratch (d.X), which
// stays in L2.  k is padded to a multiple of 16 with an identity block.
//
// One step b of the factorisation:
//   1. one wave factors the diagonal tile in registers (four columns a lane;
//      the pivot comes by readlane, each column reaches the other lanes
//      through a 64-double LDS exchange);
//   2. the panel below is solved against it, one panel row across each row
//      of 16 lanes (the solution's columns move by DPP);
//   3. every trailing tile (i, j), b < j <= i, takes A_ij -= L_ib L_jb^T with
//      four v_mfma_f64_16x16x4 (one wave a tile).
// Pivot rule: a pivot that is not finite fails; with defl == 0 (dense
// diagonal tiles) a pivot that is not positive fails, the rule of LAPACK's
// dense Cholesky factorisation; with defl > 0 a pivot <= defl
// is a dead direction whose whole column of L is zero, so the row solve
// writes a zero column of Q there.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "ktimer.h"
#include "lanes.h"

namespace tlr {
namespace {

constexpr int kT = 16;
constexpr int kTP = 17;
constexpr int kTW = kT * kTP;
constexpr int kCholLdsTiles = 11;
constexpr int kThreads = 256;
constexpr int kPanelU = 6;  // groups of four panel rows a wave solves together

typedef double v4d __attribute__((ext_vector_type(4)));

__device__ __host__ inline int tri(int i) { return i * (i + 1) / 2; }

// The largest i with tri(i) <= t (0 <= t < 2^20): the single-precision root
// is within one of it, and one select each way corrects it.
__device__ __forceinline__ int tri_root(int t) {
    int i = (int)((__builtin_amdgcn_sqrtf(8.0f * (float)t + 1.0f) - 1.0f) * 0.5f);
    i += (tri(i + 1) <= t) ? 1 : 0;
    i -= (tri(i) > t) ? 1 : 0;
    return i;
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// One wave factors diagonal tile b (wave 0 only; sets *s_fail on failure).
// Lane 16 g + r holds row r of the tile at columns g, g + 4, g + 8, g + 12,
// so the rank-one update of step c touches at most four entries a lane.
// Column c reaches the other lane groups through cbuf (64 doubles of LDS)
// while its pivot, taken by readlane from the lane that holds it, goes
// through the square root; each row below then takes
// a_rq -= (a_rc / a_cc) a_qc.  The loop has no branch, so the scheduler can
// overlap one step's updates with the next step's pivot.
__device__ __forceinline__ void diag_tile(double *TS, int b, int k, double defl, double *inv, double *cbuf,
                                          int *s_fail) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15, g = lane >> 4;
    double *D = TS + (tri(b) + b) * kTW;
    double a[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) a[s] = D[r + kTP * (4 * s + g)];
    int fail = 0;
    double my_inv = 0.0;  // 1 / L_rr, kept by lane r
#pragma unroll
    for (int c = 0; c < kT; ++c) {
        const int gc = c & 3, sc = c >> 2;  // column c sits in a[sc] of group gc
        cbuf[lane] = a[sc];
        wave_sync();
        const double xr = cbuf[16 * gc + r];  // a_rc
        double aq[4];
#pragma unroll
        for (int s = sc; s < 4; ++s) aq[s] = cbuf[16 * gc + 4 * s + g];  // a_qc, q = 4 s + g
        wave_sync();  // the next step's write follows these reads
        const double piv = readlane_d(a[sc], 16 * gc + c);
        const int gcol = kT * b + c;
        // failure or dead direction: the column is zero.  A padding column
        // (identity, untouched by the real columns) keeps its unit pivot.
        // (bitwise: no short-circuit branch in the pivot chain)
        const double ivr = rsqrt(piv);
        const bool pad = gcol >= k;
        const bool bad = !isfinite(piv) | ((defl == 0.0) & !(piv > 0.0));
        const bool zero = (bad | ((defl > 0.0) & (piv <= defl))) & !pad;
        fail = (bad & !pad & (fail == 0)) ? gcol + 1 : fail;
        const double iv = zero ? 0.0 : ivr;
        // column c of L (rows above c take values that only ever sit above
        // the diagonal, which the store zeroes); a_cc iv = sqrt(a_cc) on the
        // diagonal
        const double lrc = xr * iv;
        const double t = lrc * iv;  // a_rc / a_cc (0 for a dead direction)
        a[sc] = (g == gc) ? lrc : ((g > gc) ? a[sc] - t * aq[sc] : a[sc]);
#pragma unroll
        for (int s = sc + 1; s < 4; ++s) a[s] -= t * aq[s];
        my_inv = (r == c) ? iv : my_inv;
    }
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const int q = 4 * s + g;
        D[r + kTP * q] = (q <= r) ? a[s] : 0.0;
    }
    if (lane < kT) inv[r] = my_inv;
    if (lane == 0 && fail) *s_fail = fail;
}

// Trailing tiles t0, t0 + step, ... of step b (t numbers the tiles (i, j),
// b < j <= i, row by row from (b+1, b+1)): A_ij -= L_ib L_jb^T, two tiles at a
// time so that their operand reads and MFMA chains overlap.
__device__ __forceinline__ void trail_tiles(double *TS, int b, int count, int t0, int step) {
    const int lane = threadIdx.x & 63;
    const int li = lane & 15, lg = lane >> 4;
    auto tile_of = [&](int t, int &i, int &j) {
        const int ip = tri_root(t);
        i = b + 1 + ip;
        j = b + 1 + (t - tri(ip));
    };
#pragma unroll 1
    for (int t = t0; t < count; t += 2 * step) {
        const bool two = t + step < count;
        int i1, j1, i2, j2;
        tile_of(t, i1, j1);
        tile_of(two ? t + step : t, i2, j2);
        double *C1 = TS + (tri(i1) + j1) * kTW;
        double *C2 = TS + (tri(i2) + j2) * kTW;
        const double *L1i = TS + (tri(i1) + b) * kTW, *L1j = TS + (tri(j1) + b) * kTW;
        const double *L2i = TS + (tri(i2) + b) * kTW, *L2j = TS + (tri(j2) + b) * kTW;
        v4d acc1, acc2;
        double a1[4], b1[4], a2[4], b2[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            acc1[q] = C1[(lg + 4 * q) + kTP * li];
            acc2[q] = C2[(lg + 4 * q) + kTP * li];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            a1[s] = -L1i[li + kTP * (4 * s + lg)];
            b1[s] = L1j[li + kTP * (4 * s + lg)];
            a2[s] = -L2i[li + kTP * (4 * s + lg)];
            b2[s] = L2j[li + kTP * (4 * s + lg)];
        }
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[s], b1[s], acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a2[s], b2[s], acc2, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) C1[(lg + 4 * q) + kTP * li] = acc1[q];
        if (two) {
#pragma unroll
            for (int q = 0; q < 4; ++q) C2[(lg + 4 * q) + kTP * li] = acc2[q];
        }
    }
}

// Panel of step b: x L_bb^T = a for the 16 n rows below the diagonal tile
// (groups = 4 n groups of four rows).  Lane j of each row of 16 holds column
// j of one panel row, so column c of the solution crosses the row by DPP and
// row j of L_bb (lj, strictly lower part) stays in registers: four panel rows
// a wave instruction, U groups in flight per wave.  Lane j keeps its entry
// unscaled and scales it by ivj = 1 / L_jj once its column is done, which
// gives the same value as scaling at step j: the strictly lower row of L_bb
// leaves it unchanged afterwards.  Each entry takes the same operations in
// the same order as a row-by-row forward substitution.
template <int U, int W>
__device__ __forceinline__ void panel_rows(double *TS, int b, int groups, const double (&lj)[kT], double ivj) {
    const int tid = threadIdx.x, wave = tid >> 6;
    const int li = tid & 15, lg = (tid >> 4) & 3;
#pragma unroll 1
    for (int g0 = wave; g0 < groups; g0 += W * U) {
        double x[U];
        double *px[U];
#pragma unroll
        for (int v = 0; v < U; ++v) {
            const int g = g0 + W * v;
            const int row = 4 * (g < groups ? g : 0) + lg;  // row of the panel
            px[v] = TS + (tri(b + 1 + (row >> 4)) + b) * kTW + (row & 15) + kTP * li;
            x[v] = (g < groups) ? *px[v] : 0.0;
        }
        // each step issues its products, then its moves, then its updates,
        // U apart, so no instruction waits on the one before it (the
        // scheduler would otherwise chain the groups through one temporary)
#pragma unroll
        for (int c = 0; c < kT; ++c) {
            double m[U], xc[U];
#pragma unroll
            for (int v = 0; v < U; ++v) m[v] = x[v] * ivj;
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int v = 0; v < U; ++v) xc[v] = row_bcast_at(m[v], c);
            __builtin_amdgcn_sched_barrier(0);
#pragma unroll
            for (int v = 0; v < U; ++v) x[v] -= xc[v] * lj[c];
            __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int v = 0; v < U; ++v)
            if (g0 + W * v < groups) *px[v] = x[v] * ivj;
    }
}

// Factor the tiles in TS (tile rows T); returns the failing column + 1, or 0.
// Look-ahead: during the trailing update of step b, wave 0 updates tile
// (b+1, b+1) first and factors it at once, while the other waves update the
// rest, so each diagonal factorisation (a chain of sixteen dependent pivots)
// overlaps the previous step's updates.
template <bool LDS, int NTH>
__device__ __forceinline__ int chol_tiles(double *TS, int T, int k, double defl, double *inv, double *cbuf,
                                          int *s_fail) {
    const int tid = threadIdx.x, wave = tid >> 6;
    constexpr int kW = NTH / 64;
    if (wave == 0) diag_tile(TS, 0, k, defl, inv, cbuf, s_fail);
    __syncthreads();
    if (*s_fail) return *s_fail;
#pragma unroll 1
    for (int b = 0; b + 1 < T; ++b) {
        const int n = T - b - 1;
        // panel rows: x L_bb^T = a (panel_rows; as many groups of four rows
        // in flight per wave as the panel needs, up to kPanelU)
        {
            const int li = tid & 15;
            const double *D = TS + (tri(b) + b) * kTW;
            double lj[kT];  // row li of L_bb, strictly lower part
#pragma unroll
            for (int c = 0; c < kT; ++c) lj[c] = (c < li) ? D[li + kTP * c] : 0.0;
            const double ivj = inv[li];
            const int groups = 4 * n;
            switch ((groups + kW - 1) / kW) {
                case 1: panel_rows<1, kW>(TS, b, groups, lj, ivj); break;
                case 2: panel_rows<2, kW>(TS, b, groups, lj, ivj); break;
                case 3: panel_rows<3, kW>(TS, b, groups, lj, ivj); break;
                case 4: panel_rows<4, kW>(TS, b, groups, lj, ivj); break;
                case 5: panel_rows<5, kW>(TS, b, groups, lj, ivj); break;
                default: panel_rows<kPanelU, kW>(TS, b, groups, lj, ivj); break;
            }
        }
        __syncthreads();
        const int count = tri(n);
        if (wave == 0) {
            trail_tiles(TS, b, 1, 0, 1);  // tile (b+1, b+1)
            wave_sync();                  // its update, written across lanes, is read back by rows
            __threadfence_block();        // (tiles in global memory above 176 columns)
            diag_tile(TS, b + 1, k, defl, inv, cbuf, s_fail);
        } else {
            trail_tiles(TS, b, count, wave, kW - 1);
        }
        __syncthreads();
        if (*s_fail) return *s_fail;
    }
    return 0;
}

// Tile t of the lower triangle (row by row): (i, j) with t = i(i+1)/2 + j.
__device__ __forceinline__ void tile_rc(int t, int &i, int &j) {
    i = tri_root(t);
    j = t - tri(i);
}

// NTH threads: NTH / 256 tiles a pass, a batch of passes' loads in flight
// together.  The loads are unconditional (entries outside the lower triangle
// of the k x k matrix read A[0]) and the selects come after the batch, so no
// branch separates a load from the next one; a thread steps from one of its
// tiles to the next (TPP <= 2 further in row-by-row order) without a root.
template <bool LDS, int NTH>
__device__ __forceinline__ void load_tiles(double *TS, int T, int k, const double *A, int64_t lda, double shift) {
    constexpr int TPP = NTH / 256, BATCH = 32 / TPP;
    static_assert(TPP == 1 || TPP == 2, "one step of the tile walk covers TPP <= 2");
    const int tid = threadIdx.x;
    const int r = tid & 15, c = (tid >> 4) & 15, sub = tid >> 8;
    const int nt = tri(T);
    const int ld = (int)lda;  // k x k with k <= a few hundred: 32-bit offsets
    int ti, tj;
    tile_rc(sub, ti, tj);
#pragma unroll 1
    for (int t0 = 0; t0 < nt; t0 += BATCH * TPP) {
        double v[BATCH];
        int gr[BATCH], gc[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            gr[u] = kT * ti + r;
            gc[u] = kT * tj + c;
            const bool in = gr[u] < k && gr[u] >= gc[u];
            v[u] = A[in ? gr[u] + gc[u] * ld : 0];
            tj += TPP;
            if (tj > ti) {
                tj -= ti + 1;
                ++ti;
            }
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const int t = t0 + TPP * u + sub;
            const bool diag = gr[u] == gc[u];
            double e;
            if (gr[u] < k)
                e = (gr[u] >= gc[u]) ? v[u] + (diag ? shift : 0.0) : 0.0;
            else
                e = diag ? 1.0 : 0.0;  // identity padding
            if (t < nt) TS[t * kTW + r + kTP * c] = e;
        }
    }
}

template <int NTH>
__device__ __forceinline__ void store_r(const double *TS, int k, double *R, int64_t ldr) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int q = wave; q < k; q += NTH / 64)
        for (int r = lane; r < k; r += 64) {
            double v = 0.0;
            if (r <= q) v = TS[(tri(q >> 4) + (r >> 4)) * kTW + (q & 15) + kTP * (r & 15)];
            R[r + (int64_t)q * ldr] = v;
        }
}

constexpr int kCholThreads = 512;  // eight waves: seven update while one factors

__global__ __launch_bounds__(kCholThreads) void k_chol_small(const SmallDesc *__restrict__ descs, int mode,
                                                              DevParams *params, int lds_tiles) {
    constexpr int NTH = kCholThreads, kW = NTH / 64;
    extern __shared__ double smem[];
    const SmallDesc d = descs[blockIdx.x];
    const int k = d.k_dev ? *d.k_dev : d.k;
    if (k <= 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int T = (k + kT - 1) / kT;
    double *inv = smem + tri(lds_tiles) * kTW;
    double *cbuf = inv + kT;  // 64: the diagonal tile's column exchange
    double *red = cbuf + 64;
    int *s_fail = reinterpret_cast<int *>(red + 8);
    // mode 1: shift = 11 (m k + k (k+1)) u tr(A), and an exactly-zero panel
    // deflates instead of failing; mode 2: pivots below 1e-12 of the largest
    // diagonal entry deflate; mode 0: plain.
    double shift = 0.0, defl = 0.0;
    if (mode != 0) {
        double v = (mode == 1) ? 0.0 : 0.0;
        for (int c = tid; c < k; c += NTH) {
            const double g = d.A[c + (int64_t)c * d.lda];
            v = (mode == 1) ? v + g : fmax(v, g);
        }
        v = (mode == 1) ? wave_sum(v) : wave_max(v);
        if (lane == 0) red[wave] = v;
    }
    if (tid == 0) *s_fail = 0;
    __syncthreads();
    if (mode == 1) {
        double tr = 0.0;
#pragma unroll
        for (int w = 0; w < kW; ++w) tr += red[w];
        shift = 11.0 * ((double)d.m * k + (double)k * (k + 1)) * 1.1102230246251565e-16 * tr;
        defl = 1e-300;
    } else if (mode == 2) {
        double mx = red[0];
#pragma unroll
        for (int w = 1; w < kW; ++w) mx = fmax(mx, red[w]);
        defl = (mx > 0.0) ? 1e-12 * mx : 1e-300;
    }
    int fail;
    if (T <= lds_tiles) {
        load_tiles<true, NTH>(smem, T, k, d.A, d.lda, shift);
        __syncthreads();
        fail = chol_tiles<true, NTH>(smem, T, k, defl, inv, cbuf, s_fail);
        if (!fail) store_r<NTH>(smem, k, d.R, d.ldr);
    } else {
        load_tiles<false, NTH>(d.X, T, k, d.A, d.lda, shift);
        __syncthreads();
        fail = chol_tiles<false, NTH>(d.X, T, k, defl, inv, cbuf, s_fail);
        if (!fail) store_r<NTH>(d.X, k, d.R, d.ldr);
    }
    if (fail) {
        if (tid == 0) set_status(params, TLR_NOT_SPD, -100 - d.tile_i, -100 - d.tile_j);
        // an identity factor keeps downstream arithmetic finite
        for (int e = tid; e < k * k; e += NTH) {
            const int r = e % k, q = e / k;
            d.R[r + (int64_t)q * d.ldr] = (r == q) ? 1.0 : 0.0;
        }
    }
}

// Y (m x k, ldy) <- Y R^-1, R upper triangular (k x k, ldr), for k <= 192.  A
// work-group of four waves owns 64 rows, a wave 16 of them; the group's 64 x k
// block of Y is read into LDS once, solved there and written back once, so the
// only global reads inside the column loop are the blocks of R, each fetched
// one block ahead.  Column block b: R[0 : 16b+16, 16b : 16b+16] is staged in
// LDS; each wave takes its 16 x 16 block, subtracts X[:, :16b] R[:16b, block]
// with MFMA (X from the LDS copy, where the earlier blocks were solved), and
// solves against the diagonal block in the accumulator layout (the solution's
// columns move across each row of 16 lanes by DPP).  A zero diagonal of R
// (dead direction) gives a zero column.
constexpr int kTrsmLdsK = 192;
constexpr int kBigBatchGroups = 2048;  // eight per compute unit
constexpr int kYP = 65;  // LDS pitch of a column of the 64-row block

// kcap: the launch's largest k up to 192, padded to 16 (sizes the LDS).
__global__ __launch_bounds__(kThreads) void k_trsm_rows(const SmallDesc *__restrict__ descs, int kcap) {
    extern __shared__ double smem[];
    const SmallDesc d = descs[blockIdx.y];
    const int k = d.k_dev ? *d.k_dev : d.k;
    const int m = d.m;
    const int r0 = blockIdx.x * 64;
    if (k <= 0 || k > kcap || r0 >= m) return;
    double *Ys = smem;               // 64 x kcap, column pitch kYP
    double *Rb = smem + kYP * kcap;  // kcap x 16, row pitch kTP
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int T = (k + kT - 1) / kT;
    double *__restrict__ Y = d.Y;
    const double *__restrict__ R = d.R;
    const int64_t ldy = d.ldy, ldr = d.ldr;
    {
        const int row = r0 + (tid & 63);
        const bool rok = row < m;
        const int kp = kT * T;
        // eight columns a batch per thread (four columns a pass of the group)
#pragma unroll 1
        for (int c0 = 0; c0 < kp; c0 += 32) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int col = c0 + 4 * u + (tid >> 6);
                v[u] = (rok && col < k) ? Y[row + (int64_t)col * ldy] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int col = c0 + 4 * u + (tid >> 6);
                if (col < kp) Ys[col * kYP + (tid & 63)] = v[u];
            }
        }
    }
    const int wr = kT * wave;  // this wave's first row in the block
    __shared__ double invd[kT];
    // R block b, R[0 : 16b+16, 16b : 16b+16], goes through registers: its
    // loads are issued one block ahead, behind the current block's arithmetic
    constexpr int kRv = kTrsmLdsK / kT;
    double rv[kRv];
    auto load_r = [&](int b) {
        const int rows = kT * b + kT;
#pragma unroll
        for (int u = 0; u < kRv; ++u) {
            const int e = tid + kThreads * u, q = e >> 4, j = e & 15, gc = kT * b + j;
            rv[u] = (q < rows && q < k && gc < k) ? R[q + (int64_t)gc * ldr] : ((q == gc) ? 1.0 : 0.0);
        }
    };
    load_r(0);
    for (int b = 0; b < T; ++b) {
        __syncthreads();  // Ys loaded / the previous block's Rb consumed
        {
            const int rows = kT * b + kT;
#pragma unroll
            for (int u = 0; u < kRv; ++u) {
                const int e = tid + kThreads * u, q = e >> 4, j = e & 15;
                if (q < rows) Rb[q * kTP + j] = rv[u];
                if (q == kT * b + j) invd[j] = (rv[u] != 0.0) ? 1.0 / rv[u] : 0.0;
            }
        }
        __syncthreads();
        if (b + 1 < T) load_r(b + 1);
        const int col = kT * b + li;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] = Ys[col * kYP + wr + lg + 4 * q];
        // 4b K-steps of four (a multiple of four), four at a time into four
        // independent partial sums, so consecutive MFMAs do not wait on each
        // other; the partial sums join the block at the end
        const int ns = 4 * b;
        v4d part[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) part[u] = v4d{0.0, 0.0, 0.0, 0.0};
        for (int s0 = 0; s0 < ns; s0 += 4) {
            double av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int kap = 4 * (s0 + u) + lg;
                av[u] = Ys[kap * kYP + wr + li];
                bv[u] = Rb[kap * kTP + li];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) part[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], part[u], 0, 0, 0);
        }
        if (ns > 0) acc -= (part[0] + part[1]) + (part[2] + part[3]);
        // diagonal block: x R_bb = y for the wave's 16 rows in the
        // accumulator layout (lane li holds column li of rows lg + 4 q), so
        // column j of the solution crosses the row by DPP while row j of
        // R_bb (strictly upper part) stays in registers.  Lane li keeps its
        // entry unscaled and scales it once its column is done: the same
        // operations, in the same order, as a row-by-row substitution.
        {
            const double *Rd = Rb + (kT * b) * kTP;  // rows 16b.. of the staged block
            double rj[kT];
#pragma unroll
            for (int j = 0; j < kT; ++j) rj[j] = (j < li) ? Rd[j * kTP + li] : 0.0;
            const double ivl = invd[li];
#pragma unroll
            for (int j = 0; j < kT; ++j) {
                double mm[4], xc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) mm[q] = acc[q] * ivl;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) xc[q] = row_bcast_at(mm[q], j);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] -= xc[q] * rj[j];
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] *= ivl;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) Ys[col * kYP + wr + lg + 4 * q] = acc[q];
    }
    __syncthreads();
    {
        const int row = r0 + (tid & 63);
        if (row < m)
#pragma unroll 4
            for (int col = tid >> 6; col < k; col += 4) Y[row + (int64_t)col * ldy] = Ys[col * kYP + (tid & 63)];
    }
}

// The same with Y read from and written to global memory (the earlier
// blocks' X is read back from Y), for every k above k_lo: k > 192, or all k
// in batches too large for one LDS-bound work-group per compute unit.
__global__ __launch_bounds__(kThreads) void k_trsm_rows_wide(const SmallDesc *__restrict__ descs, int k_lo) {
    extern __shared__ double Rb[];
    const SmallDesc d = descs[blockIdx.y];
    const int k = d.k_dev ? *d.k_dev : d.k;
    const int m = d.m;
    const int r0 = blockIdx.x * 64;
    if (k <= k_lo || r0 >= m) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lg = lane >> 4;
    const int rowbase = r0 + kT * wave;
    const int T = (k + kT - 1) / kT;
    double *__restrict__ Y = d.Y;
    const double *__restrict__ R = d.R;
    const int64_t ldy = d.ldy, ldr = d.ldr;
    for (int b = 0; b < T; ++b) {
        __syncthreads();
        const int rows = kT * b + kT;
        for (int e = tid; e < rows * kT; e += kThreads) {
            const int q = e >> 4, j = e & 15, gc = kT * b + j;
            Rb[q * kTP + j] = (q < k && gc < k) ? R[q + (int64_t)gc * ldr] : ((q == gc) ? 1.0 : 0.0);
        }
        __syncthreads();
        const int col = kT * b + li;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rowbase + lg + 4 * q;
            acc[q] = (row < m && col < k) ? Y[row + (int64_t)col * ldy] : 0.0;
        }
        const int arow = rowbase + li;
        const bool arow_ok = arow < m;
        // eight K-steps at a time: their operand loads are issued together
        for (int s0 = 0; s0 < 4 * b; s0 += 8) {
            double av[8], bv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int kap = 4 * (s0 + u) + lg;
                const bool in = s0 + u < 4 * b;
                av[u] = (in && arow_ok) ? -Y[arow + (int64_t)kap * ldy] : 0.0;
                bv[u] = in ? Rb[kap * kTP + li] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (s0 + u < 4 * b) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
        // diagonal block as in k_trsm_rows: column j crosses the row by DPP,
        // lane li scales its entry once its column is done
        {
            const double *Rd = Rb + (kT * b) * kTP;  // rows 16b.. of the staged block
            double rj[kT];
#pragma unroll
            for (int j = 0; j < kT; ++j) rj[j] = (j < li) ? Rd[j * kTP + li] : 0.0;
            const double rll = Rd[li * kTP + li];
            const double ivl = (rll != 0.0) ? 1.0 / rll : 0.0;
#pragma unroll
            for (int j = 0; j < kT; ++j) {
                double mm[4], xc[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) mm[q] = acc[q] * ivl;
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) xc[q] = row_bcast_at(mm[q], j);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int q = 0; q < 4; ++q) acc[q] -= xc[q] * rj[j];
                __builtin_amdgcn_sched_barrier(0);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[q] *= ivl;
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rowbase + lg + 4 * q;
            if (row < m && col < k) Y[row + (int64_t)col * ldy] = acc[q];
        }
    }
}

// Cholesky of one bs x bs diagonal block A[b0:b0+bs, b0:b0+bs] (ld) of a
// dense diagonal tile, in LDS with the tile algorithm above (plain pivots: a
// pivot <= 0 fails with TLR_NOT_SPD for the tile).
__global__ __launch_bounds__(kThreads) void k_potrf_block(double *A, int ld, int b0, int bs, int tile,
                                                           DevParams *params) {
    constexpr int TB = 4;  // 64 = 4 tiles
    __shared__ double ts[(TB * (TB + 1) / 2) * kTW];
    __shared__ double inv[kT];
    __shared__ double cbuf[64];
    __shared__ int s_fail;
    if (params->status != 0) return;
    const int tid = threadIdx.x;
    if (tid == 0) s_fail = 0;
    const int T = (bs + kT - 1) / kT;
    double *Ab = A + b0 + (int64_t)b0 * ld;
    load_tiles<true, kThreads>(ts, T, bs, Ab, ld, 0.0);
    __syncthreads();
    const int fail = chol_tiles<true, kThreads>(ts, T, bs, 0.0, inv, cbuf, &s_fail);
    if (fail) {
        if (tid == 0) set_status(params, TLR_NOT_SPD, tile, tile);
        return;
    }
    for (int e = tid; e < bs * bs; e += kThreads) {
        const int r = e % bs, q = e / bs;
        if (r >= q) Ab[r + (int64_t)q * ld] = ts[(tri(r >> 4) + (q >> 4)) * kTW + (r & 15) + kTP * (q & 15)];
    }
}

// Rows r in [b0+bs, nrows): A[r, b0:b0+bs] <- A[r, b0:b0+bs] L_bb^-T, one row
// per thread.
__global__ __launch_bounds__(kThreads) void k_potrf_panel(double *A, int ld, int b0, int bs, int nrows,
                                                           DevParams *params) {
    __shared__ double L[64 * 65];
    const int tid = threadIdx.x;
    if (params->status != 0) return;
    {
        // sixteen loads a thread, all in flight together
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + kThreads * u, r = e & 63, q = e >> 6;
            v[u] = (r < bs && q < bs && r >= q) ? A[(b0 + r) + (int64_t)(b0 + q) * ld] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e = tid + kThreads * u, r = e & 63, q = e >> 6;
            L[r + q * 65] = v[u];
        }
    }
    __syncthreads();
    const int row = b0 + bs + blockIdx.x * kThreads + tid;
    if (row >= nrows) return;
    double x[64];
#pragma unroll
    for (int c = 0; c < 64; ++c) x[c] = (c < bs) ? A[row + (int64_t)(b0 + c) * ld] : 0.0;
    // column-oriented: once x_c is final it is taken out of every later
    // entry, which sees the same subtractions in the same order as a row dot
    // product would give it, with a far shorter dependent chain
#pragma unroll
    for (int c = 0; c < 64; ++c) {
        if (c < bs) {
            const double xc = x[c] / L[c + c * 65];
            x[c] = xc;
#pragma unroll
            for (int cq = c + 1; cq < 64; ++cq) x[cq] -= xc * L[cq + c * 65];
        }
    }
#pragma unroll
    for (int c = 0; c < 64; ++c)
        if (c < bs) A[row + (int64_t)(b0 + c) * ld] = x[c];
}

}  // namespace

tlr_status potrf_tile(double *A, int nb, int tile, DevParams *params, const GemmDesc *d_desc, hipStream_t s) {
    static const int cls_b = ktimer_class("k_potrf_block"), cls_p = ktimer_class("k_potrf_panel");
    const int nblk = (int)cdiv(nb, 64);
    for (int b = 0; b < nblk; ++b) {
        const int b0 = b * 64, bs = (nb - b0 < 64) ? nb - b0 : 64;
        const int rest = nb - b0 - bs;
        {
            const double d = bs;
            KTimer kt(cls_b, s, d * d * d / 3.0, 8.0 * d * (d + 1.0), true);
            hipLaunchKernelGGL(k_potrf_block, dim3(1), dim3(kThreads), 0, s, A, nb, b0, bs, tile, params);
        }
        if (rest > 0) {
            {
                const double d = bs, r = rest;
                KTimer kt(cls_p, s, r * d * d, 8.0 * (2.0 * r * d + d * (d + 1.0) / 2.0), true);
                hipLaunchKernelGGL(k_potrf_panel, dim3((unsigned)cdiv(rest, kThreads)), dim3(kThreads), 0, s, A, nb,
                                   b0, bs, nb, params);
            }
            // the trailing update: only its lower triangle is ever read
            TLR_TRY(gemm_batched(false, true, d_desc + b, 1, rest, rest, s, nullptr, true));
        }
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status chol_small(const SmallDesc *d_descs, int count, int max_k, int mode, DevParams *params,
                      hipStream_t s, const SmallDesc *h_descs) {
    if (count <= 0 || max_k <= 0) return TLR_OK;
    if (max_k > kMaxSketch) return TLR_E_UNSUPPORTED;
    static const int cls = ktimer_class("k_chol_small");
    static const bool attr = [] {
        return hipFuncSetAttribute(reinterpret_cast<const void *>(k_chol_small),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024) == hipSuccess;
    }();
    if (!attr) (void)hipGetLastError();  // launches above 64 KB will then report the limit
    (void)attr;
    double flops = 0.0, bytes = 0.0;
    if (h_descs && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const double k = h_descs[t].k;
            flops += k * k * k / 3.0;
            bytes += 8.0 * k * (k + 1.0);  // lower triangle in, upper factor out
        }
    const int tmax = (max_k + kT - 1) / kT;
    const int lds_tiles = tmax < kCholLdsTiles ? tmax : kCholLdsTiles;
    const size_t lds = sizeof(double) * ((size_t)tri(lds_tiles) * kTW + kT + 64 + 8) + 16;
    KTimer kt(cls, s, flops, bytes, h_descs != nullptr);
    hipLaunchKernelGGL(k_chol_small, dim3(count), dim3(kCholThreads), lds, s, d_descs, mode, params, lds_tiles);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status trsm_rows(const SmallDesc *d_descs, int count, int max_m, int max_k, hipStream_t s,
                     const SmallDesc *h_descs) {
    if (count <= 0 || max_m <= 0 || max_k <= 0) return TLR_OK;
    if (max_k > kMaxSketch) return TLR_E_UNSUPPORTED;
    static const int cls = ktimer_class("k_trsm_rows"), cls_w = ktimer_class("k_trsm_rows_wide");
    static const bool attr = [] {
        const bool a = hipFuncSetAttribute(reinterpret_cast<const void *>(k_trsm_rows),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024) == hipSuccess;
        const bool b = hipFuncSetAttribute(reinterpret_cast<const void *>(k_trsm_rows_wide),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024) == hipSuccess;
        return a && b;
    }();
    if (!attr) (void)hipGetLastError();  // launches above 64 KB will then report the limit
    (void)attr;
    double flops = 0.0, bytes = 0.0, flops_w = 0.0, bytes_w = 0.0;
    if (h_descs && ktimer_on())
        for (int t = 0; t < count; ++t) {
            const double k = h_descs[t].k, m = h_descs[t].m;
            const double f = m * k * k, b = 8.0 * (2.0 * m * k + k * (k + 1.0) / 2.0);
            if (h_descs[t].k <= kTrsmLdsK) {
                flops += f;
                bytes += b;
            } else {
                flops_w += f;
                bytes_w += b;
            }
        }
    const dim3 grid((unsigned)cdiv(max_m, 64), (unsigned)count);
    // The LDS-resident kernel holds one or two work-groups per compute unit;
    // it pays off while the batch is a few work-groups per unit (a column of
    // the factorisation, at most 99 panels of 15 row blocks).  Larger batches
    // (a compression wave) keep every unit busy with the global-memory kernel.
    const bool big = (int64_t)grid.x * grid.y > kBigBatchGroups;
    int k_lo = kTrsmLdsK;
    if (big) {
        k_lo = 0;
        flops_w += flops;
        bytes_w += bytes;
    } else {
        const int kcap = (std::min(max_k, kTrsmLdsK) + kT - 1) / kT * kT;
        const size_t lds = sizeof(double) * ((size_t)kYP * kcap + (size_t)kcap * kTP);
        KTimer kt(cls, s, flops, bytes, h_descs != nullptr);
        hipLaunchKernelGGL(k_trsm_rows, grid, dim3(kThreads), lds, s, d_descs, kcap);
    }
    if (max_k > k_lo) {
        const int kp = (max_k + kT - 1) / kT * kT;
        const size_t lds = sizeof(double) * (size_t)kp * kTP;
        KTimer kt(cls_w, s, flops_w, bytes_w, h_descs != nullptr);
        hipLaunchKernelGGL(k_trsm_rows_wide, grid, dim3(kThreads), lds, s, d_descs, k_lo);
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
