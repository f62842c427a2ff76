// Host-side launchers of the library's device kernels.
#pragma once

#include "common.h"
#include "matern.h"

namespace tlr {

// One product C = alpha * op(A) * op(B) + beta * C of a batched launch.
// Matrices are column-major.  op(A) is M x K, op(B) is K x N.  When an
// override pointer is set, the device value replaces the field (sizes that
// are only known on the device, e.g. a rank computed by an earlier kernel).
struct GemmDesc {
    const void *A;  // element type of A, B and C: see the `types` bits below
    const void *B;
    void *C;
    const int32_t *M_dev;
    const int32_t *N_dev;
    const int32_t *K_dev;
    int32_t M, N, K;
    int32_t lda, ldb, ldc;
    double alpha, beta;
};

// trans_a / trans_b: op(X) = X^T.  max_m, max_n bound every product's M, N
// (they size the grid; products smaller than the bound exit early).
// h_descs: optional host copy of the descriptors, used only to count the
// launch's work for the launch timer.
// types: which of A, B, C hold float32 (the rest float64); the arithmetic is
// float64 in every case.  Supported: none, C, A, A+B, A+C, B+C.
enum { kGemmA32 = 1, kGemmB32 = 2, kGemmC32 = 4 };
tlr_status gemm_batched(bool trans_a, bool trans_b, const GemmDesc *d_descs, int count, int max_m,
                        int max_n, hipStream_t s, const GemmDesc *h_descs = nullptr,
                        bool lower_only = false, int types = 0);

// Small dense problems, one work-group each.
struct SmallDesc {
    double *A;        // k x k input (lda)
    double *R;        // k x k output (ldr)
    double *X;        // k x k output: left singular vectors (ldx)
    double *S;        // k output: singular values
    double *Y;        // m x k panel (ldy) for the row solves
    int32_t *rank;    // out: rank at tol (Jacobi)
    int32_t *flag;    // out: 1 if the sketch was too narrow (Jacobi)
    const int32_t *k_dev;  // optional device k
    int32_t k, lda, ldr, ldx, m, ldy;
    int32_t k_full;        // sketch width at which the sample is exact
    int32_t tile_i, tile_j;
    // mixed precision: extra rounding-noise norm of the tile's operator (a
    // device value added to ||A||_F in the truncation floor), or null
    const double *noise;
};

// R = upper Cholesky factor of A (+ shift I).  mode 1: shift = 11 (m k +
// k(k+1)) u trace(A); mode 2: no shift, pivots below 1e-12 max diag(A) deflate
// their column; mode 0: plain.  A is read-only.
tlr_status chol_small(const SmallDesc *d_descs, int count, int max_k, int mode, DevParams *params,
                      hipStream_t s, const SmallDesc *h_descs = nullptr);
// Y <- Y R^-1 (R upper triangular k x k), in place, row by row.
tlr_status trsm_rows(const SmallDesc *d_descs, int count, int max_m, int max_k, hipStream_t s,
                     const SmallDesc *h_descs = nullptr);
// Largest sketch width any kernel accepts.
constexpr int kMaxSketch = 512;

// One-sided Jacobi SVD of A (k x k): S descending, X = left singular vectors,
// R = k x k scratch (used when k is too large for LDS),
// rank = #{S > tol}; flag = 1 when fewer than `min_tail` values are <= tol
// and k < k_full (the sample was too narrow to resolve the threshold).
tlr_status jacobi_svd(const SmallDesc *d_descs, int count, int max_k, double tol, int min_tail,
                      int k_full, int rank_cap, DevParams *params, hipStream_t s);

// Truncated Householder QR with column pivoting of A (k x k): rank r is the
// first step whose trailing Frobenius norm is <= thr, where thr = tol, or
// with params->floor_rel > 0 (factors stored in float32)
// thr = max(tol, floor_rel (||A||_F + *noise)); X = Q1 (k x r),
// Y = B^T (k x r) with A ~ Q1 B; R = k x k scratch (when k is too large for LDS).
// flag = 1 (rank 0 written) when k - r < min_tail and k < k_full.
tlr_status qrcp_trunc(const SmallDesc *d_descs, int count, int max_k, double tol, int min_tail, int k_full,
                      int rank_cap, DevParams *params, hipStream_t s,
                      int min_k = 1);

// Dense diagonal-tile kernels (nb x nb, column-major, ld = nb).
// Blocked Cholesky (block 64): the trailing updates use ceil(nb/64) GEMM
// descriptors built by potrf_tile_descs and staged on the device by the caller.
void potrf_tile_descs(double *A, int nb, GemmDesc *h);
tlr_status potrf_tile(double *A, int nb, int tile, DevParams *params, const GemmDesc *d_desc, hipStream_t s);

struct CopyDesc {
    const void *src;
    void *dst;
    int64_t words;
    int32_t conv;  // 0: float64 -> float64, 1: float32 -> float64, 2: float32 -> float32
};
tlr_status copy_batched(const CopyDesc *d_descs, int count, int64_t max_words, hipStream_t s);
// Host resources the library keeps in pools for the life of the process
// (pinned staging buffers, streams), counted where they are created.
void note_pinned_alloc();
void note_stream_created();
void alloc_counts(int64_t *pinned, int64_t *streams);
// Each of the `count` nb x nb matrices (device pointer array) set to I.
tlr_status identity_batched(double *const *d_ptrs, int count, int nb, hipStream_t s);
// B_t <- L^-1 B_t for `count` right-hand-side panels (nb x cols_t, ld nb),
// L lower (nb x nb).  descs: A = L (shared), Y = B_t, k = cols_t.
// d_gemm / h_gemm: room for count * ceil(nb/64) descriptors; h_gemm ==
// nullptr means the caller has already put them at d_gemm (see below).
// y32: the panels hold float32 (read and written as such; float64 arithmetic).
tlr_status trsm_left_lower(const double *L, int nb, const SmallDesc *d_descs, const SmallDesc *h_descs,
                           int count, int max_cols, GemmDesc *d_gemm, GemmDesc *h_gemm, hipStream_t s,
                           bool y32 = false);
// The GEMM descriptors trsm_left_lower uses (ceil(nb/64) * count entries,
// block major), for a caller that uploads them itself.
void trsm_left_lower_descs(const double *L, int nb, const SmallDesc *h_descs, int count, GemmDesc *h_gemm,
                           bool y32 = false);

// Matern tile generation.
struct GenDesc {
    double *dst;        // nb x nb, column-major, ld
    int32_t row0, col0; // global start indices
    int32_t ld;
    int32_t diag;       // 1 for a diagonal tile
};
tlr_status gen_tiles_launch(const GenDesc *d_descs, int count, int nb, int64_t n, const double *x,
                            const double *y, const MaternConst &c, hipStream_t s);

// Per-theta table for general nu (kChebPieces * (kChebDeg+1) doubles at tab);
// sets c->tab (left null for the closed forms).
tlr_status build_knu_table(MaternConst *c, double *tab, hipStream_t s);
// Bivariate model: n is the matrix size (twice the number of locations in x, y).
tlr_status gen_tiles_biv_launch(const GenDesc *d_descs, int count, int nb, int64_t n, const double *x,
                                const double *y, const BivConst &c, hipStream_t s);

// Misc.
tlr_status gaussian_fill(double *out, int64_t count, uint64_t seed, hipStream_t s);
tlr_status split_locs(const double *locs, int64_t n, int64_t npad, double *x, double *y, hipStream_t s);
tlr_status pad_copy(const double *z, int64_t n, int64_t npad, double *out, hipStream_t s);
// y = Li z for one nb x nb lower-triangular inverse Li (column-major), out of
// place; skipped once the status word records a failure.
tlr_status tri_gemv(const double *Li, int nb, const double *z, double *y, const DevParams *params, hipStream_t s);
size_t gemv_desc_bytes();
void make_gemv_desc(void *dst, const void *U, const void *V, const double *yj, double *yi,
                    const int32_t *r_dev);
// f32: U and V of every descriptor hold float32.
tlr_status lr_gemv(const void *d_descs, int count, int nb, const DevParams *params, hipStream_t s,
                   bool f32 = false);
// Frobenius norms of low-rank factor panels (nb x r float32, r from the
// device): out[t] = ||V_t||_F.  One work-group a panel.
struct NormDesc {
    const float *V;
    const int32_t *r_dev;
    double *out;
};
tlr_status factor_norms(const NormDesc *d_descs, int count, int nb, hipStream_t s);
// Rounding-noise norm of the Schur complement of tile (i, j) at column j:
// out[t] = sqrt(nrm_s[i nt + j]^2 + sum_{k<j} (nrm_l[i nt + k] nrm_l[j nt + k])^2).
struct NoiseDesc {
    int32_t i, j;
    double *out;
};
tlr_status schur_noise(const NoiseDesc *d_descs, int count, int nt, const double *nrm_s, const double *nrm_l,
                       hipStream_t s);
tlr_status logdet_quad(const double *diag, int nb, int nt, int64_t n, const double *yv, const DevParams *params,
                       double *out, hipStream_t s);
// dst[:, c] = src[:, c] for c < *cols_dev (rows x cols panels).
tlr_status copy_panel(const double *src, int64_t lds, double *dst, int64_t ldd, int rows, const int32_t *cols_dev,
                      int max_cols, hipStream_t s);

// Tukey g-and-h: z = tau^-1((t - xi)/omega) elementwise; then
// out[3] = sum log(omega tau'(z_i)) and out[2] -= out[3] (-inf if not finite).
tlr_status tgh_inverse(const double *t, int64_t n, double xi, double omega, double g, double h, double *z,
                       hipStream_t s);
tlr_status tgh_combine(const double *z, int64_t n, double omega, double g, double h, double *out, hipStream_t s);

// Attainable peaks (measured): streaming copy bandwidth and FP64 MFMA rate.
tlr_status peak_hbm(const void *src, void *dst, int64_t bytes, int reps, double *gbs, hipStream_t s);
tlr_status peak_mfma_f64(double *scratch, int64_t scratch_words, int iters, double *tflops, hipStream_t s);

// Orderings.
size_t reorder_ws_bytes(int64_t n, tlr_ordering kind);
tlr_status reorder(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                   int32_t *d_perm, void *d_ws, size_t ws_bytes, hipStream_t s);
tlr_status reorder_noalloc(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                           int32_t *d_perm, hipStream_t s);
int64_t reorder_noalloc_max_n();
tlr_status apply_perm(const int32_t *d_perm, int64_t n, const double *d_locs, const double *d_z,
                      double *d_locs_out, double *d_z_out, int dequant, hipStream_t s);

}  // namespace tlr
