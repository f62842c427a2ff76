// Matern tile generation, the sketch test matrix, and the TLR forward solve
// with the log-determinant / quadratic-form reductions.
#include <algorithm>
#include <cmath>

#include "kernels.h"
#include "ktimer.h"

namespace tlr {

bool make_matern_const(double sigma2, double beta, double nu, MaternConst *out) {
    if (!(sigma2 > 0.0) || !(beta > 0.0) || !(nu > 0.0)) return false;
    if (!std::isfinite(sigma2) || !std::isfinite(beta) || !std::isfinite(nu)) return false;
    if (nu > 60.0) return false;
    MaternConst c{};
    c.sigma2 = sigma2;
    c.beta = beta;
    c.nu = nu;
    c.kind = (nu == 0.5) ? 1 : (nu == 1.5) ? 2 : (nu == 2.5) ? 3 : 0;
    const int N = (int)std::floor(nu + 0.5);
    const double mu = nu - (double)N;
    c.N = N;
    c.mu = mu;
    c.coef = sigma2 / (std::tgamma(nu) * std::pow(2.0, nu - 1.0));
    const long double gp = std::tgamma(1.0L + (long double)mu);
    const long double gm = std::tgamma(1.0L - (long double)mu);
    c.gp = (double)gp;
    c.gm = (double)gm;
    c.gam2 = (double)(0.5L * (1.0L / gm + 1.0L / gp));
    if (std::fabs(mu) < 0.05) {
        // odd Taylor coefficients of 1/Gamma(1+z) (Abramowitz & Stegun 6.1.34)
        const double m2 = mu * mu;
        c.gam1 = -(0.57721566490153286061 +
                   m2 * (-0.042002635034095235529 +
                         m2 * (-0.042197734555544336748 +
                               m2 * (0.0072189432466630995424 +
                                     m2 * (-0.00021524167411495097282 + m2 * -0.000020134854780788238656)))));
    } else {
        c.gam1 = (double)((1.0L / gm - 1.0L / gp) / (2.0L * (long double)mu));
    }
    c.fact = (mu == 0.0) ? 1.0 : (double)((long double)mu * 3.14159265358979323846264338327950288L /
                                          std::sin((long double)mu * 3.14159265358979323846264338327950288L));
    *out = c;
    return true;
}

bool make_biv_const(double s11, double s22, double a, double nu11, double nu22, double beta12, BivConst *out) {
    if (!std::isfinite(beta12) || !(std::fabs(beta12) <= 1.0)) return false;
    const double nu12 = 0.5 * (nu11 + nu22);
    BivConst b{};
    if (!make_matern_const(s11, a, nu11, &b.m[0]) || !make_matern_const(s22, a, nu22, &b.m[2]) ||
        !make_matern_const(1.0, a, nu12, &b.m[1]))
        return false;
    // colocated correlation of the cited parsimonious model in two
    // dimensions: beta_12 sqrt(Gamma(nu11+1)/Gamma(nu11) Gamma(nu22+1)/Gamma(nu22))
    // Gamma(nu12)/Gamma(nu12+1) = beta_12 sqrt(nu11 nu22) / nu12
    const double rho = beta12 * std::sqrt(nu11 * nu22) / nu12;
    const double scale = rho * std::sqrt(s11 * s22);
    b.m[1].sigma2 = scale;
    b.m[1].coef *= scale;
    b.on = 1;
    *out = b;
    return true;
}

namespace {

// One work-group per (tile, group of 8 columns): threads run down the rows,
// so the stores of a column are contiguous.  KIND is the Matern branch
// (1: nu=1/2, 2: nu=3/2, 3: nu=5/2, 0: general nu), fixed per instantiation so
// the closed forms do not carry the register footprint of the K_nu code.
template <int KIND>
__device__ inline double matern_kind(double d, const MaternConst &c) {
    const double x = d / c.beta;
    if (KIND == 1) return c.sigma2 * exp(-x);
    if (KIND == 2) return c.sigma2 * (1.0 + x) * exp(-x);
    if (KIND == 3) return c.sigma2 * (1.0 + x + x * x / 3.0) * exp(-x);
    if (x == 0.0) return c.sigma2;
    if (x > kTabXhi) return 0.0;
    if (x < kTabXlo || c.tab == nullptr) return c.coef * xnu_knu(x, c);
    return c.coef * xnu_knu_tab(x, c);
}

// Chebyshev coefficients of h on each piece from its kChebDeg+1 Chebyshev
// nodes of the first kind (one work-group per piece).
__global__ __launch_bounds__(64) void k_knu_table(MaternConst c, double *tab) {
    __shared__ double f[kChebDeg + 1];
    const int piece = blockIdx.x, j = threadIdx.x;
    const int n1 = kChebDeg + 1;
    const double w = 1.0 / c.inv_w;
    const double mid = c.s_lo + (piece + 0.5) * w, half = 0.5 * w;
    if (j < n1) {
        const double t = cos(3.14159265358979323846 * (j + 0.5) / n1);
        f[j] = log_xnu_knu_scaled(exp(mid + half * t), c);
    }
    __syncthreads();
    if (j < n1) {
        double acc = 0.0;
        for (int q = 0; q < n1; ++q) acc += f[q] * cos(3.14159265358979323846 * j * (q + 0.5) / n1);
        acc *= 2.0 / n1;
        if (j == 0) acc *= 0.5;
        tab[piece * n1 + j] = acc;
    }
}

template <int KIND>
__global__ __launch_bounds__(256) void k_gen_tiles(const GenDesc *__restrict__ descs, int nb, int64_t n,
                                                   const double *__restrict__ x, const double *__restrict__ y,
                                                   MaternConst c) {
    const GenDesc d = descs[blockIdx.y];
    const int q0 = blockIdx.x * 8;
    for (int q = q0; q < q0 + 8 && q < nb; ++q) {
        const int64_t gj = d.col0 + q;
        const bool jin = gj < n;
        const double xj = jin ? x[gj] : 0.0, yj = jin ? y[gj] : 0.0;
        double *col = d.dst + (int64_t)q * d.ld;
        for (int r = threadIdx.x; r < nb; r += blockDim.x) {
            const int64_t gi = d.row0 + r;
            double v;
            if (gi >= n || !jin) {
                v = (gi == gj) ? 1.0 : 0.0;  // identity padding of the ragged last tile
            } else if (gi == gj) {
                v = c.sigma2;
            } else {
                const double dx = x[gi] - xj, dy = y[gi] - yj;
                v = matern_kind<KIND>(sqrt(dx * dx + dy * dy), c);
            }
            col[r] = v;
        }
    }
}

// C(d) of one function with its kind chosen at run time (the bivariate
// generator mixes three functions in one tile).
__device__ inline double matern_any(double d, const MaternConst &c) {
    switch (c.kind) {
        case 1: return matern_kind<1>(d, c);
        case 2: return matern_kind<2>(d, c);
        case 3: return matern_kind<3>(d, c);
        default: return matern_kind<0>(d, c);
    }
}

// Bivariate tiles: entry (gi, gj) of the 2n x 2n matrix is C_{v w}(|s_p - s_q|)
// with p = gi / 2, v = gi % 2, q = gj / 2, w = gj % 2.  x, y hold the n
// locations; `n` here is the matrix size 2n.
__global__ __launch_bounds__(256) void k_gen_tiles_biv(const GenDesc *__restrict__ descs, int nb, int64_t n,
                                                       const double *__restrict__ x, const double *__restrict__ y,
                                                       BivConst bc) {
    const GenDesc d = descs[blockIdx.y];
    const int q0 = blockIdx.x * 8;
    for (int q = q0; q < q0 + 8 && q < nb; ++q) {
        const int64_t gj = d.col0 + q;
        const bool jin = gj < n;
        const int64_t pj = gj >> 1;
        const int wj = (int)(gj & 1);
        const double xj = jin ? x[pj] : 0.0, yj = jin ? y[pj] : 0.0;
        double *col = d.dst + (int64_t)q * d.ld;
        for (int r = threadIdx.x; r < nb; r += blockDim.x) {
            const int64_t gi = d.row0 + r;
            double v;
            if (gi >= n || !jin) {
                v = (gi == gj) ? 1.0 : 0.0;  // identity padding of the ragged last tile
            } else {
                const MaternConst &c = bc.m[(int)(gi & 1) + wj];
                const int64_t pi = gi >> 1;
                if (pi == pj) {
                    v = c.sigma2;  // colocated: the variance, or rho_12 sigma_11 sigma_22
                } else {
                    const double dx = x[pi] - xj, dy = y[pi] - yj;
                    v = matern_any(sqrt(dx * dx + dy * dy), c);
                }
            }
            col[r] = v;
        }
    }
}

// Counter-based standard normals: SplitMix64 pairs -> Box-Muller.
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_gaussian(double *out, int64_t count, uint64_t seed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint64_t a = mix64(seed + (2 * (uint64_t)i + 1) * 0x9E3779B97F4A7C15ull);
    const uint64_t b = mix64(seed + (2 * (uint64_t)i + 2) * 0x9E3779B97F4A7C15ull);
    const double u1 = ((double)(a >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);
    out[i] = sqrt(-2.0 * log(u1)) * cospi(2.0 * u2);
}

__global__ void k_split_locs(const double *__restrict__ locs, int64_t n, int64_t npad, double *__restrict__ x,
                             double *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    x[i] = (i < n) ? locs[2 * i] : 0.0;
    y[i] = (i < n) ? locs[2 * i + 1] : 0.0;
}

__global__ void k_pad_copy(const double *__restrict__ z, int64_t n, int64_t npad, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npad) out[i] = (i < n) ? z[i] : 0.0;
}

// y = L^-1 z for one diagonal tile, with L^-1 (lower triangular, nb x nb,
// column-major) formed during the factorisation: a product, out of place.
// A work-group owns 32 rows and splits the columns up to its last row 32
// ways (thread g of a row takes c = g, g + 32, ...; four partial sums a
// thread), then adds the 32 partials of each row in a fixed order, so the
// result is the same on every call.  Columns past a row are exact zeros of
// L^-1 and add nothing.
constexpr int kTgRows = 32, kTgSplit = 32, kTgThreads = kTgRows * kTgSplit;
__global__ __launch_bounds__(kTgThreads) void k_tri_gemv(const double *__restrict__ Li, int nb,
                                                          const double *__restrict__ z, double *__restrict__ y,
                                                          const DevParams *params) {
    __shared__ double zs[4096];
    __shared__ double part[kTgSplit][kTgRows];
    if (params->status != 0) return;
    const int r0 = blockIdx.x * kTgRows;
    const int tid = threadIdx.x, rr = tid % kTgRows, g = tid / kTgRows;
    const int r = r0 + rr;
    const int cend = (nb < r0 + kTgRows) ? nb : r0 + kTgRows;
    for (int c = tid; c < cend; c += kTgThreads) zs[c] = z[c];
    __syncthreads();
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    if (r < nb) {
        const double *__restrict__ row = Li + r;
        int c = g;
        for (; c + 3 * kTgSplit < cend; c += 4 * kTgSplit) {
            a0 += row[(int64_t)c * nb] * zs[c];
            a1 += row[(int64_t)(c + kTgSplit) * nb] * zs[c + kTgSplit];
            a2 += row[(int64_t)(c + 2 * kTgSplit) * nb] * zs[c + 2 * kTgSplit];
            a3 += row[(int64_t)(c + 3 * kTgSplit) * nb] * zs[c + 3 * kTgSplit];
        }
        for (; c < cend; c += kTgSplit) a0 += row[(int64_t)c * nb] * zs[c];
    }
    part[g][rr] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    if (g == 0 && r < nb) {
        double acc = part[0][rr];
#pragma unroll 8
        for (int q = 1; q < kTgSplit; ++q) acc += part[q][rr];
        y[r] = acc;
    }
}

struct GemvDesc {
    const void *U;  // float64, or float32 in the f32 instantiation
    const void *V;
    const double *yj;
    double *yi;
    const int32_t *r_dev;
};

// y_i <- y_i - U (V^T y_j) for a batch of low-rank tiles (one work-group each).
// Both products are latency-bound on a single work-group, so every loop keeps
// a batch of independent loads in flight: y_j is read into registers once,
// a wave forms two dot products V[:, c]^T y_j at a time, and each thread
// updates its four rows of y_i from four columns of U at a time.
constexpr int kGemvRowsPerLane = 16;  // nb <= 1024 in registers; longer tiles loop

template <class T>
__global__ __launch_bounds__(256) void k_lr_gemv(const GemvDesc *__restrict__ descs, int nb,
                                                 const DevParams *params) {
    __shared__ double t[4096];  // rank <= nb <= 4096 (a dense tile has rank nb)
    const GemvDesc d = descs[blockIdx.x];
    const T *__restrict__ Uf = static_cast<const T *>(d.U);
    const T *__restrict__ Vf = static_cast<const T *>(d.V);
    const int r = *d.r_dev;
    if (r <= 0 || params->status != 0) return;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int q0 = 0; q0 < nb; q0 += 64 * kGemvRowsPerLane) {
        double yj[kGemvRowsPerLane];
#pragma unroll
        for (int u = 0; u < kGemvRowsPerLane; ++u) {
            const int q = q0 + lane + 64 * u;
            yj[u] = (q < nb) ? d.yj[q] : 0.0;
        }
        for (int c = wave; c < r; c += 8) {
            const int c2 = c + 4;
            const T *v1 = Vf + (int64_t)c * nb;
            const T *v2 = Vf + (int64_t)(c2 < r ? c2 : c) * nb;
            double a1 = 0.0, a2 = 0.0;
            // every load of the two columns issued before the first use (a
            // float32 entry is widened only at its multiply); rows past the
            // tile read its last row, which meets yj = 0 there
            T w1[kGemvRowsPerLane], w2[kGemvRowsPerLane];
#pragma unroll
            for (int u = 0; u < kGemvRowsPerLane; ++u) {
                const int q = min(q0 + lane + 64 * u, nb - 1);
                w1[u] = v1[q];
                w2[u] = v2[q];
            }
#pragma unroll
            for (int u = 0; u < kGemvRowsPerLane; ++u) {
                a1 += (double)w1[u] * yj[u];
                a2 += (double)w2[u] * yj[u];
            }
            for (int off = 32; off > 0; off >>= 1) {
                a1 += __shfl_xor(a1, off, 64);
                a2 += __shfl_xor(a2, off, 64);
            }
            if (lane == 0) {
                t[c] = (q0 == 0) ? a1 : t[c] + a1;
                if (c2 < r) t[c2] = (q0 == 0) ? a2 : t[c2] + a2;
            }
        }
    }
    __syncthreads();
    for (int row0 = tid; row0 < nb; row0 += 4 * 256) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int c = 0;
        for (; c + 4 <= r; c += 4) {
            T uv[4][4];
            // rows past the tile read its last row; their sums are never stored
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int row = min(row0 + 256 * k, nb - 1);
                    uv[k][w] = Uf[row + (int64_t)(c + w) * nb];
                }
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[k] += (double)uv[k][w] * t[c + w];
        }
        for (; c < r; ++c)
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int row = row0 + 256 * k;
                if (row < nb) acc[k] += (double)Uf[row + (int64_t)c * nb] * t[c];
            }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int row = row0 + 256 * k;
            if (row < nb) d.yi[row] -= acc[k];
        }
    }
}

// out = {logdet, quad, loglik}; fixed-order reduction (bitwise reproducible).
__global__ __launch_bounds__(1024) void k_logdet_quad(const double *__restrict__ diag, int nb, int nt, int64_t n,
                                                      const double *__restrict__ yv, const DevParams *params,
                                                      double *__restrict__ out) {
    __shared__ double s_ld[1024], s_q[1024];
    const int tid = threadIdx.x;
    double ld = 0.0, q = 0.0;
    for (int64_t i = tid; i < n; i += 1024) {
        const int64_t k = i / nb, r = i % nb;
        ld += log(diag[k * (int64_t)nb * nb + r + r * (int64_t)nb]);
        q += yv[i] * yv[i];
    }
    s_ld[tid] = ld;
    s_q[tid] = q;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (tid < s) {
            s_ld[tid] += s_ld[tid + s];
            s_q[tid] += s_q[tid + s];
        }
        __syncthreads();
    }
    if (tid == 0) {
        const double logdet = 2.0 * s_ld[0];
        const double quad = s_q[0];
        out[0] = logdet;
        out[1] = quad;
        const double ll = -0.5 * (double)n * 1.8378770664093454836 - 0.5 * logdet - 0.5 * quad;
        out[2] = (params->status != 0 || !isfinite(ll)) ? -INFINITY : ll;
    }
    (void)nt;
}

}  // namespace

tlr_status gen_tiles_launch(const GenDesc *d_descs, int count, int nb, int64_t n, const double *x,
                            const double *y, const MaternConst &c, hipStream_t s) {
    if (count <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_gen_tiles");
    // every tile is written once in full (padding included); the locations
    // it reads are a rounding error beside that
    KTimer kt(cls, s, 0.0, 8.0 * (double)nb * nb * count, true);
    const dim3 grid((unsigned)cdiv(nb, 8), count), block(256);
    switch (c.kind) {
        case 1: hipLaunchKernelGGL(k_gen_tiles<1>, grid, block, 0, s, d_descs, nb, n, x, y, c); break;
        case 2: hipLaunchKernelGGL(k_gen_tiles<2>, grid, block, 0, s, d_descs, nb, n, x, y, c); break;
        case 3: hipLaunchKernelGGL(k_gen_tiles<3>, grid, block, 0, s, d_descs, nb, n, x, y, c); break;
        default: hipLaunchKernelGGL(k_gen_tiles<0>, grid, block, 0, s, d_descs, nb, n, x, y, c); break;
    }
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status gen_tiles_biv_launch(const GenDesc *d_descs, int count, int nb, int64_t n, const double *x,
                                const double *y, const BivConst &c, hipStream_t s) {
    if (count <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_gen_tiles");
    KTimer kt(cls, s, 0.0, 8.0 * (double)nb * nb * count, true);
    const dim3 grid((unsigned)cdiv(nb, 8), count), block(256);
    hipLaunchKernelGGL(k_gen_tiles_biv, grid, block, 0, s, d_descs, nb, n, x, y, c);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status build_knu_table(MaternConst *c, double *tab, hipStream_t s) {
    c->tab = nullptr;
    c->nint = kChebPieces;
    c->s_lo = std::log(kTabXlo);
    c->inv_w = kChebPieces / (std::log(kTabXhi) - std::log(kTabXlo));
    if (c->kind != 0) return TLR_OK;
    hipLaunchKernelGGL(k_knu_table, dim3(kChebPieces), dim3(64), 0, s, *c, tab);
    TLR_HIP(hipGetLastError());
    c->tab = tab;
    return TLR_OK;
}

tlr_status gaussian_fill(double *out, int64_t count, uint64_t seed, hipStream_t s) {
    if (count <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_gaussian, dim3((unsigned)cdiv(count, 256)), dim3(256), 0, s, out, count, seed);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status split_locs(const double *locs, int64_t n, int64_t npad, double *x, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_split_locs, dim3((unsigned)cdiv(npad, 256)), dim3(256), 0, s, locs, n, npad, x, y);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status pad_copy(const double *z, int64_t n, int64_t npad, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_pad_copy, dim3((unsigned)cdiv(npad, 256)), dim3(256), 0, s, z, n, npad, out);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

namespace {
__global__ __launch_bounds__(256) void k_identity(double *const *__restrict__ ptrs, int nb) {
    double *V = ptrs[blockIdx.y];
    const int words = nb * nb;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < words; e += gridDim.x * 256)
        V[e] = (e % nb == e / nb) ? 1.0 : 0.0;
}
}  // namespace

tlr_status identity_batched(double *const *d_ptrs, int count, int nb, hipStream_t s) {
    if (count <= 0 || nb <= 0) return TLR_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv((int64_t)nb * nb, 256), 1024);
    hipLaunchKernelGGL(k_identity, dim3(gx, count), dim3(256), 0, s, d_ptrs, nb);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status tri_gemv(const double *Li, int nb, const double *z, double *y, const DevParams *params, hipStream_t s) {
    if (nb > 4096) return TLR_E_UNSUPPORTED;
    static const int cls = ktimer_class("k_tri_gemv");
    const double b = nb;
    KTimer kt(cls, s, b * (b + 1.0), 8.0 * (b * (b + 1.0) / 2.0 + 2.0 * b), true);
    hipLaunchKernelGGL(k_tri_gemv, dim3((unsigned)cdiv(nb, kTgRows)), dim3(kTgThreads), 0, s, Li, nb, z, y, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

tlr_status lr_gemv(const void *d_descs, int count, int nb, const DevParams *params, hipStream_t s, bool f32) {
    if (count <= 0) return TLR_OK;
    static const int cls = ktimer_class("k_lr_gemv");
    KTimer kt(cls, s, 0.0, 0.0, false);  // ranks live in the descriptors on the device
    if (f32)
        hipLaunchKernelGGL((k_lr_gemv<float>), dim3(count), dim3(256), 0, s, static_cast<const GemvDesc *>(d_descs),
                           nb, params);
    else
        hipLaunchKernelGGL((k_lr_gemv<double>), dim3(count), dim3(256), 0, s, static_cast<const GemvDesc *>(d_descs),
                           nb, params);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

size_t gemv_desc_bytes() { return sizeof(GemvDesc); }

void make_gemv_desc(void *dst, const void *U, const void *V, const double *yj, double *yi,
                    const int32_t *r_dev) {
    GemvDesc g{U, V, yj, yi, r_dev};
    *static_cast<GemvDesc *>(dst) = g;
}

tlr_status logdet_quad(const double *diag, int nb, int nt, int64_t n, const double *yv, const DevParams *params,
                       double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_logdet_quad, dim3(1), dim3(1024), 0, s, diag, nb, nt, n, yv, params, out);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

namespace {
__global__ void k_copy_panel(const double *__restrict__ src, int64_t lds_, double *__restrict__ dst,
                             int64_t ldd, int rows, const int32_t *cols_dev) {
    const int cols = *cols_dev;
    const int c = blockIdx.y;
    if (c >= cols) return;
    for (int r = blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += gridDim.x * blockDim.x)
        dst[r + c * ldd] = src[r + c * lds_];
}
}  // namespace

tlr_status copy_panel(const double *src, int64_t lds_, double *dst, int64_t ldd, int rows, const int32_t *cols_dev,
                      int max_cols, hipStream_t s) {
    if (max_cols <= 0) return TLR_OK;
    hipLaunchKernelGGL(k_copy_panel, dim3((unsigned)cdiv(rows, 256), max_cols), dim3(256), 0, s, src, lds_, dst,
                       ldd, rows, cols_dev);
    TLR_HIP(hipGetLastError());
    return TLR_OK;
}

}  // namespace tlr
