/*
 * tlrmle.h -- C ABI of the MI355X tile-low-rank Matern log-likelihood library.
 *
 * The library evaluates the Gaussian log-likelihood
 *     l(theta) = -(n/2) log(2 pi) - (1/2) log|Sigma(theta)| - (1/2) Z^T Sigma(theta)^-1 Z
 * (paper Section 1, eq. "loglik") for the Matern covariance of Section 4.1
 * (eq. "maternkernel"), theta = (sigma2, beta, nu), after the locations have
 * been reordered (Section 3), through a tile low-rank (TLR) Cholesky
 * factorisation of Sigma (Section 2).
 *
 * Conventions shared by every call:
 *  - Pointers named d_* are device (HBM) pointers owned by the caller; h_*
 *    are host pointers owned by the caller.  The library never keeps a
 *    reference to them after the call returns (except d_ws between calls of
 *    one evaluation, see below).
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call that takes a stream is asynchronous on it unless stated.
 *  - Argument errors are detected on the host before any launch and returned
 *    as TLR_E_* codes; nothing is enqueued in that case.  Numerical failures
 *    (a non-positive pivot, a tile rank above the cap) are written by the
 *    kernels to a status word inside the workspace (first failure wins) and
 *    surface as l = -infinity; read them with tlr_status_read().
 *  - Layouts: locations are n x 2 float64, array-of-structs (x0, y0, x1, ...);
 *    matrices are column-major.
 *  - No global mutable state: calls on different workspaces may run
 *    concurrently from different host threads.
 */
#ifndef TLRMLE_H
#define TLRMLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tlr_status;

enum {
    TLR_OK = 0,
    TLR_E_INVAL = 1,        /* bad argument (null pointer, size, theta <= 0, NaN) */
    TLR_E_NOMEM = 2,        /* workspace smaller than the queried size */
    TLR_E_UNSUPPORTED = 3,  /* combination not implemented */
    TLR_E_HIP = 4,          /* a HIP runtime call failed */
    TLR_NOT_SPD = 16,       /* device: non-positive pivot in a diagonal tile */
    TLR_RANK_OVERFLOW = 17, /* device: a tile rank exceeded the plan's rank cap */
    TLR_E_DOMAIN = 18,      /* device: a location outside [0,1]^2 or not finite */
    TLR_ARENA_OVERFLOW = 19 /* the factors outgrew the workspace's rank budget */
};

/* Orderings of paper Section 3: NONE = generation order ("No Order"),
 * RANDOM = seeded permutation, MORTON / HILBERT = space-filling-curve keys of
 * the 16-bit encoded coordinates (Sections 3.1.1, 3.1.2), KDTREE = in-order
 * leaves of the median-split KD-tree (Section 3.2). */
typedef enum {
    TLR_ORDER_NONE = 0,
    TLR_ORDER_RANDOM = 1,
    TLR_ORDER_MORTON = 2,
    TLR_ORDER_HILBERT = 3,
    TLR_ORDER_KDTREE = 4
} tlr_ordering;

/* Arithmetic of the factorisation.  FP64 everywhere, or low-rank factors and
 * off-diagonal products in FP32 (diagonal-tile Cholesky, log-determinant and
 * quadratic-form reductions stay FP64). */
typedef enum {
    TLR_FP64 = 0,
    TLR_MIXED_FP32 = 1
} tlr_precision;

/* Matern parameters (paper eq. "maternkernel"): variance, range, smoothness. */
typedef struct {
    double sigma2;
    double beta;
    double nu;
} tlr_theta;

/* Device status, read back by tlr_status_read(). */
typedef struct {
    int32_t code;       /* TLR_OK or the first TLR_NOT_SPD / TLR_RANK_OVERFLOW */
    int32_t tile_i;     /* tile row of the first failure (-1 if none) */
    int32_t tile_j;     /* tile column of the first failure (-1 if none) */
    int32_t max_rank;   /* largest off-diagonal rank held by the factor */
    int64_t rank_sum;   /* sum of off-diagonal ranks held by the factor */
} tlr_devinfo;

/* flags for tlr_reorder */
#define TLR_REORDER_DEQUANTIZE 1u /* also write code/65535 coordinates (decoding step) */

/* flags for tlr_plan_create */
#define TLR_PLAN_DEFAULT 0u
/* Keep an off-diagonal tile whose rank exceeds maxrank dense instead of
 * failing (the paper's dense fallback, Section 2 / Table "memory").  The
 * workspace then holds one nb x nb pair per off-diagonal tile besides the
 * low-rank slots. */
#define TLR_PLAN_DENSE_TILES 1u
/* Truncation rule of every compression and recompression (Section 2's
 * accuracy threshold tol, absolute):
 *  - default: pivoted QR of the projected k x k factor, stopped at the first
 *    step whose trailing Frobenius norm is <= tol.  The spectral error is
 *    <= tol; the rank is at or a few above the singular-value count.
 *  - TLR_PLAN_SVD_TRUNCATION: one-sided Jacobi SVD of that factor, rank =
 *    #{singular values > tol} -- the paper's rule exactly (slower).
 * The rule is a property of the plan; the d_ranks output of tlr_compress
 * only reports the ranks the rule produced. */
#define TLR_PLAN_SVD_TRUNCATION 2u

typedef struct tlr_plan_s *tlr_plan;
typedef struct tlr_batch_plan_s *tlr_batch_plan;

/* ------------------------------------------------------------------------ */
/* Ordering (paper Section 3)                                                */
/* ------------------------------------------------------------------------ */

/* Device workspace bytes tlr_reorder needs for n points of the given kind. */
size_t tlr_reorder_ws_bytes(int64_t n, tlr_ordering kind);

/* Ordering permutation.
 * d_locs: n x 2 float64 AoS, every coordinate in [0,1] (Section 3.1's unit
 *         square); outside values set TLR_E_DOMAIN in the returned status
 *         after a synchronous check (this call synchronises `stream` once).
 * kind:   see tlr_ordering.  MORTON/HILBERT encode each coordinate as
 *         rint(x * 65535) (ties to even) -- the "Encoding" step -- build the
 *         32-bit curve key and sort by (key, original index) -- the "Sorting"
 *         step.  RANDOM sorts by the SplitMix64 stream started at `seed`.
 *         KDTREE splits on the larger-range coordinate at the median, first
 *         ceil(m/2) points (by coordinate, then index) to the left.
 * d_perm: out, n int32: d_perm[k] = original index of the k-th ordered point.
 * d_ws:   caller workspace of at least tlr_reorder_ws_bytes(n, kind) bytes.
 * The result is bit-identical to the paper-derived CPU definition. */
tlr_status tlr_reorder(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed,
                       uint32_t flags, int32_t *d_perm, void *d_ws, size_t ws_bytes, void *stream);

/* Allocation-free tlr_reorder, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments and bit-identical result as
 * tlr_reorder, without a workspace: the ordering runs in a scratch array of
 * fixed size that the library holds on every device it runs on, from its
 * load to the end of the process.  Nothing is allocated or freed.
 * n <= tlr_reorder_noalloc_max_n() (131,072 points); a larger n returns
 * TLR_E_NOMEM before anything is enqueued.  All calls on one device share
 * that device's scratch array: calls that overlap on one device (two host
 * threads, or two streams without an ordering between them) race and give
 * undefined results; serialise them.  The scratch keeps whatever the last
 * call left; every call rewrites all it reads. */
tlr_status tlr_reorder_noalloc(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed,
                               uint32_t flags, int32_t *d_perm, void *stream);
int64_t tlr_reorder_noalloc_max_n(void);

/* Gather locations (n x 2 AoS) and observations by d_perm:
 * d_locs_out[k] = d_locs[d_perm[k]], d_z_out[k] = d_z[d_perm[k]].
 * With dequantize != 0 the gathered coordinates are rint(x*65535)/65535
 * (the "Decoding" step of Section 3.1).  d_z / d_z_out may be NULL. */
tlr_status tlr_apply_perm(const int32_t *d_perm, int64_t n, const double *d_locs, const double *d_z,
                          double *d_locs_out, double *d_z_out, int32_t dequantize, void *stream);

/* ------------------------------------------------------------------------ */
/* Plan and workspace                                                        */
/* ------------------------------------------------------------------------ */

/* Host-only, immutable description of one problem shape.
 * n >= 1 points, tile size nb >= 16 (nt = ceil(n/nb) tiles per side; a
 * ragged last tile is padded with identity rows/columns and zero
 * observations, which leaves log|Sigma| and the quadratic form unchanged).
 * maxrank: cap on an off-diagonal tile rank; <= 0 means nb/2 (the storage
 * break-even of Section 3).  A tile whose rank exceeds the cap stops the
 * factorisation with TLR_RANK_OVERFLOW (the "cannot proceed" case of
 * Section 3.3 / Table "memory"), unless flags has TLR_PLAN_DENSE_TILES: then
 * the tile is kept dense (stored as the pair U = tile, V = I of rank nb) and
 * the factorisation goes on.
 * Allocates host memory only. */
tlr_status tlr_plan_create(tlr_plan *out, int64_t n, int32_t nb, int32_t maxrank,
                           tlr_precision precision, uint32_t flags);
void tlr_plan_destroy(tlr_plan plan);

/* Bytes of device workspace one evaluation needs: a fixed part (diagonal
 * tiles and their inverses, sketch and small-matrix buffers, descriptors,
 * tables, status word)
 * and a factor arena that holds the low-rank factors U, V of every
 * off-diagonal tile in slots of 2 * nb * w entries (w >= the tile's rank;
 * 8-byte entries, 4-byte in a TLR_MIXED_FP32 plan).
 * rank_budget: the total of the slot widths w the arena must hold (the sum of
 * the off-diagonal ranks, plus the growth of tiles whose rank rises in the
 * factorisation); <= 0 means maxrank for every tile, which always suffices.
 * A smaller budget sizes admission by the ranks a problem really has; if the
 * factors outgrow it, the evaluation stops with TLR_ARENA_OVERFLOW (l = -inf).
 * Every call takes the caller's workspace size and uses all of it: a larger
 * buffer is a larger arena.  The library never allocates device memory on the
 * evaluation path. */
size_t tlr_plan_ws_bytes(tlr_plan plan, int64_t rank_budget);

/* Tile geometry of the plan (any pointer may be NULL). */
void tlr_plan_shape(tlr_plan plan, int64_t *n, int32_t *nb, int32_t *nt, int32_t *maxrank);

/* ------------------------------------------------------------------------ */
/* The hot path, step by step (an evaluation is gen -> compress -> potrf ->  */
/* solve_logdet on one workspace; tlr_loglik runs all four)                  */
/* ------------------------------------------------------------------------ */

/* Covariance generation (eqs. "covfunc", "maternkernel"):
 * diagonal tiles Sigma_kk written densely into the workspace, and the
 * locations + theta recorded for the off-diagonal tiles, which are generated
 * on demand by tlr_compress.  d_locs: ordered n x 2 AoS.  Resets the device
 * status word. */
tlr_status tlr_gen_tiles(tlr_plan plan, const double *d_locs, tlr_theta theta, void *d_ws,
                         size_t ws_bytes, void *stream);

/* Compression (Section 2, Fig. "tlr"; Section 3's accuracy threshold):
 * every off-diagonal tile A_ij (i > j) becomes U_ij V_ij^T with
 * ||A_ij - U_ij V_ij^T||_2 <= tol (absolute threshold), by a randomised range
 * finder with one power step and the plan's truncation rule applied to the
 * small projected matrix (see TLR_PLAN_SVD_TRUNCATION).  d_ranks: optional
 * out, nt*nt int32 (row-major, entry i*nt + j for i > j; other entries 0):
 * the rank of each tile, -1 when it exceeded maxrank (then the status word
 * is TLR_RANK_OVERFLOW), -2 when it is kept dense.  Requesting d_ranks does
 * not change the computation. */
tlr_status tlr_compress(tlr_plan plan, double tol, void *d_ws, size_t ws_bytes, int32_t *d_ranks,
                        void *stream);

/* TLR Cholesky factorisation Sigma~ = L L^T, in place in the workspace.
 * Left-looking by tile column: the Schur complement of each off-diagonal
 * tile is re-compressed once at the plan's tol; diagonal tiles are factored
 * densely in FP64, and each column's panel factors V_ij are multiplied by
 * the explicit inverse of L_jj, formed beside the recompression on a second
 * stream of default priority and kept in the workspace for
 * tlr_solve_logdet.  A non-positive pivot sets TLR_NOT_SPD (tile k, k).
 * Host-synchronises `stream` once per tile column (ranks are read back to
 * size the next column's work). */
tlr_status tlr_potrf(tlr_plan plan, void *d_ws, size_t ws_bytes, void *stream);

/* Forward solve y = L^-1 Z, log|Sigma~| = 2 sum log L_ii, quad = y^T y, in
 * FP64, after tlr_potrf on the same workspace (the diagonal blocks of the
 * solve are products with the inverses it kept).  d_z: ordered observations,
 * n float64.  d_out: out, 3 float64 on the
 * device: {logdet, quad, loglik}; loglik = -inf when the status is not OK. */
tlr_status tlr_solve_logdet(tlr_plan plan, const double *d_z, void *d_ws, size_t ws_bytes,
                            double *d_out, void *stream);

/* One evaluation: gen_tiles -> compress -> potrf -> solve_logdet.
 * d_out as for tlr_solve_logdet.  d_ranks as for tlr_compress (may be NULL). */
tlr_status tlr_loglik(tlr_plan plan, const double *d_locs, const double *d_z, tlr_theta theta,
                      double tol, void *d_ws, size_t ws_bytes, double *d_out, int32_t *d_ranks,
                      void *stream);

/* ------------------------------------------------------------------------ */
/* Parsimonious bivariate Matern model (Section 4.2.1, eq. "bivmatern")      */
/* ------------------------------------------------------------------------ */

/* Two variables at the same n locations; one range a, marginal variances and
 * smoothnesses, cross smoothness nu_12 = (nu_11 + nu_22)/2 and colocated
 * correlation rho_12 = beta_12 sqrt(nu_11 nu_22) / nu_12 (the cited
 * definition's Gamma ratios in two dimensions).  Valid for |beta_12| <= 1. */
typedef struct {
    double sigma2_11;
    double sigma2_22;
    double a;
    double nu_11;
    double nu_22;
    double beta_12;
} tlr_theta_biv;

/* As tlr_gen_tiles for the 2n x 2n bivariate covariance.  The plan's n is the
 * matrix size (even): d_locs holds n/2 ordered locations (n/2 x 2 AoS) and
 * matrix entry 2p + v belongs to variable v (0 or 1) at location p.  The
 * following tlr_compress / tlr_potrf / tlr_solve_logdet calls on the same
 * workspace use this model.  TLR_E_INVAL for an odd n or an invalid theta. */
tlr_status tlr_gen_tiles_bivariate(tlr_plan plan, const double *d_locs, tlr_theta_biv theta, void *d_ws,
                                   size_t ws_bytes, void *stream);

/* One bivariate evaluation: tlr_gen_tiles_bivariate -> compress -> potrf ->
 * solve_logdet.  d_z: n observations, location-major (d_z[2p + v] = Z_v(s_p)).
 * d_out, d_ranks as for tlr_loglik. */
tlr_status tlr_loglik_bivariate(tlr_plan plan, const double *d_locs, const double *d_z, tlr_theta_biv theta,
                                double tol, void *d_ws, size_t ws_bytes, double *d_out, int32_t *d_ranks,
                                void *stream);

/* ------------------------------------------------------------------------ */
/* Tukey g-and-h random fields (Section 4.2.2)                              */
/* ------------------------------------------------------------------------ */

/* T(s) = xi + omega tau(Z(s)), tau(z) = g^-1 (exp(g z) - 1) exp(h z^2 / 2)
 * (g = 0: z exp(h z^2 / 2)), Z a standard Gaussian random field.  Valid
 * parameters: xi, g finite, omega > 0, h >= 0 (tau is then increasing). */
typedef struct {
    double xi;
    double omega;
    double g;
    double h;
} tlr_tgh;

/* d_z[i] = tau^-1((d_t[i] - xi) / omega), i < n: the Gaussian observation
 * behind each TGH observation, in float64 (closed form when h = 0, else
 * bracketed Newton iteration to a few ulps).  A value with no preimage
 * (h = 0 and g (t - xi)/omega <= -1) or not finite gives NaN.  d_t and d_z
 * may alias.  n = 0 is a no-op.  TLR_E_INVAL for invalid parameters. */
tlr_status tlr_tgh_inverse(const double *d_t, int64_t n, tlr_tgh p, double *d_z, void *stream);

/* TGH log-likelihood by the change of variables:
 *     l_TGH = l(theta; z) - sum_i log(omega tau'(z_i)),  z = tlr_tgh_inverse(t),
 * l(theta; z) the TLR Gaussian log-likelihood of tlr_loglik (theta of the
 * Gaussian field: sigma2 = 1 for the standard field of the model).  d_t:
 * ordered observations, n = the plan's n; d_z: out, n float64 (the
 * transformed observations); d_out: out, 4 float64 on the device:
 * {logdet, quad, l_TGH, sum_i log(omega tau'(z_i))}; l_TGH = -inf when the
 * status is not OK or some observation has no preimage. */
tlr_status tlr_loglik_tgh(tlr_plan plan, const double *d_locs, const double *d_t, tlr_theta theta, tlr_tgh p,
                          double tol, void *d_ws, size_t ws_bytes, double *d_z, double *d_out, void *stream);

/* ------------------------------------------------------------------------ */
/* Batched evaluation of independent problems                               */
/* ------------------------------------------------------------------------ */

/* One plan per problem (count >= 1; h_n[p] points, tile size h_nb[p]; the
 * same maxrank, precision and flags for all), as tlr_plan_create.  Host-only.
 * The batch workspace is the problems' workspaces back to back. */
tlr_status tlr_batch_plan_create(tlr_batch_plan *out, int32_t count, const int64_t *h_n, const int32_t *h_nb,
                                 int32_t maxrank, tlr_precision precision, uint32_t flags);
void tlr_batch_plan_destroy(tlr_batch_plan bplan);
size_t tlr_batch_ws_bytes(tlr_batch_plan bplan);

/* l(theta_p) of every problem p of the batch: the evaluation of tlr_loglik
 * for each (Section 1 eq. "loglik" through Sections 2-4), run on `workers`
 * (1..16) library-owned streams of default priority, widest problems first,
 * so that the problems' small factorisation kernels overlap on the device.
 * h_locs, h_z: host arrays of count device pointers (ordered n_p x 2 AoS
 * locations and n_p observations); h_theta: host array of count thetas.
 * d_out: device, count x 3 float64 ({logdet, quad, loglik} per problem, as
 * tlr_solve_logdet; loglik = -inf for a problem whose status is not OK).
 * Work queued on `stream` before the call is finished before any problem
 * starts; `stream` waits for every problem's work.  The call returns once
 * every problem has been issued (each evaluation synchronises its own
 * stream per tile column, as tlr_potrf does).  Results are bitwise those of
 * tlr_loglik on each problem alone.  Batched calls on one device are
 * serialised by the library. */
tlr_status tlr_loglik_batched(tlr_batch_plan bplan, const double *const *h_locs, const double *const *h_z,
                              const tlr_theta *h_theta, double tol, void *d_ws, size_t ws_bytes, double *d_out,
                              int32_t workers, void *stream);

/* tlr_status_read for problem `index` of a batch (synchronises `stream`). */
tlr_status tlr_batch_status_read(tlr_batch_plan bplan, const void *d_ws, int32_t index, tlr_devinfo *out,
                                 void *stream);

/* Synchronises `stream`, then reads the device status word. */
/* Per-tile ranks held in the workspace: which = 0 gives those of Sigma's
 * compressed tiles (after tlr_compress), which = 1 those of the factor L
 * (after tlr_potrf).  d_out: device, nt*nt int32, row-major, entry (i, j)
 * for i > j (other entries 0; -1 marks a tile whose rank exceeded maxrank,
 * -2 a tile kept dense under TLR_PLAN_DENSE_TILES).
 * Synchronises `stream`.  (Paper Section 5.2: per-tile ranks and the
 * storage they imply.) */
tlr_status tlr_ranks_read(tlr_plan plan, const void *d_ws, int32_t which, int32_t *d_out, void *stream);

tlr_status tlr_status_read(tlr_plan plan, const void *d_ws, tlr_devinfo *out, void *stream);

/* Human-readable name of a status code (static string). */
const char *tlr_strerror(tlr_status code);

/* Version string of the library build. */
const char *tlr_version(void);

/* ------------------------------------------------------------------------ */
/* Launch timer                                                              */
/* ------------------------------------------------------------------------ */

/* Per-kernel statistics of the launches made while the timer is on.  Each
 * instrumented launch is bracketed by two HIP events on the stream it runs
 * on; `total_ms` sums their elapsed times.  `flops` and `bytes` are the
 * algorithmic work of the launches whose sizes are known on the host
 * (`exact_launches`, taking `exact_ms`): operations the method needs, and
 * each operand read and each result written once in HBM.  Names are kernel
 * function names as a profiler's kernel trace shows them (template
 * arguments abbreviated). */
typedef struct tlr_kstat {
    char name[48];
    int64_t launches;
    double total_ms;
    int64_t exact_launches;
    double exact_ms;
    double flops;
    double bytes;
} tlr_kstat;

/* Turn the timer on (nonzero) or off.  Timing adds two event records per
 * launch; it does not synchronise the stream. */
tlr_status tlr_kstats_enable(int32_t on);
/* Restrict timing to the kernel class called `name` (the name
 * tlr_kstats_read reports, e.g. "k_chol_small"); NULL or "" times every
 * class again.  Launches of other classes then carry no events at all, which
 * keeps the timer's own cost off the untimed kernels.  Unknown names are
 * registered (and then match nothing until such a kernel runs). */
tlr_status tlr_kstats_select(const char *name);
/* Wait for pending timed launches, then zero every counter. */
tlr_status tlr_kstats_reset(void);
/* Wait for pending timed launches and copy up to `max` entries into `out`
 * (host array).  Returns the number of kernel classes (may exceed `max`),
 * or -1 when `out` is null and `max` > 0. */
int32_t tlr_kstats_read(tlr_kstat *out, int32_t max);

/* ------------------------------------------------------------------------ */
/* Kernel diagnostics (used by the test suite to check the building blocks)  */
/* ------------------------------------------------------------------------ */

/* C = alpha op(A) op(B) + beta C on the float64 matrix-core GEMM used by
 * every sketch product and update above.  Column-major device matrices;
 * op(X) = X^T when trans_x != 0.  op(A) is M x K, op(B) is K x N.  With
 * beta == 0, C is not read.  Synchronises `stream`; allocates and frees a
 * one-descriptor device temporary (diagnostic use only). */
tlr_status tlr_diag_gemm(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K, double alpha,
                         const double *d_A, int32_t lda, const double *d_B, int32_t ldb, double beta,
                         double *d_C, int32_t ldc, void *stream);

/* `count` products of one shape in one batched launch, C_t = alpha op(A_t)
 * op(B_t) + beta C_t with X_t = d_X + t * stride_x (elements): the launch the
 * likelihood path makes for a batch of tile products, including its choice
 * between the K-split kernel and the LDS-staged kernel for tall batches (at
 * least 256 rows of C and 256 row blocks of 64 over the batch).
 * count <= 65535.  Synchronises `stream`; allocates and frees a descriptor
 * temporary (diagnostic use only). */
tlr_status tlr_diag_gemm_strided(int32_t trans_a, int32_t trans_b, int32_t count, int32_t M, int32_t N, int32_t K,
                                 double alpha, const double *d_A, int32_t lda, int64_t stride_a, const double *d_B,
                                 int32_t ldb, int64_t stride_b, double beta, double *d_C, int32_t ldc,
                                 int64_t stride_c, void *stream);

/* Attainable peaks of the two roofs the evaluation is measured against,
 * timed with HIP events on `stream` (synchronises it).
 * tlr_diag_peak_hbm: `reps` streaming copies d_src -> d_dst of `bytes`
 * bytes each (16-byte aligned device buffers); *h_gbs = bytes read plus
 * bytes written per second / 1e9.
 * tlr_diag_peak_mfma_f64: independent v_mfma_f64_16x16x4 chains, `iters`
 * steps on eight waves of every compute unit; *h_tflops = FP64 matrix-core
 * flops per second / 1e12.  d_scratch receives one double per thread
 * (scratch_words >= 512 * compute units). */
tlr_status tlr_diag_peak_hbm(const void *d_src, void *d_dst, int64_t bytes, int32_t reps, double *h_gbs,
                             void *stream);
tlr_status tlr_diag_peak_mfma_f64(double *d_scratch, int64_t scratch_words, int32_t iters, double *h_tflops,
                                  void *stream);

/* Host resources the library has created in this process and keeps in pools
 * for reuse: *h_pinned pinned host staging buffers, *h_streams streams (side
 * streams of the factorisation, batch worker streams).  Both counts stop
 * growing once every pool has reached the size a workload needs, so a count
 * that still grows across repeated evaluations would mean an allocation per
 * evaluation.  The library makes no device allocation on the evaluation path
 * (the workspace is the caller's).  TLR_E_INVAL for a null pointer. */
tlr_status tlr_diag_alloc_counts(int64_t *h_pinned, int64_t *h_streams);

/* Copy tile (i, j) of the matrix held in the workspace into d_out (nb x nb,
 * column-major): for i == j the dense diagonal tile (Sigma_jj after
 * tlr_gen_tiles, its Cholesky factor in the lower triangle after tlr_potrf);
 * for i > j the product U_ij V_ij^T of the stored low-rank factors (the
 * compressed Sigma_ij after tlr_compress, L_ij after tlr_potrf).  *h_rank
 * (may be NULL) receives the tile's rank (nb for a diagonal tile).
 * Synchronises `stream`. */
tlr_status tlr_diag_tile(tlr_plan plan, const void *d_ws, int32_t i, int32_t j, double *d_out, int32_t *h_rank,
                         void *stream);

/* Orthonormalise an m x k panel by the CholeskyQR passes of the compression
 * step (two shifted passes, two deflating passes): on return d_Y holds Q
 * (m x k, ld m; a zero column marks a direction below rounding) and d_R the
 * k x k upper-triangular factor with Y_in = Q R.  k <= 512.  d_scratch: at
 * least 512 + 7*8*k*k bytes.  Synchronises `stream`. */
tlr_status tlr_diag_cholqr(int32_t m, int32_t k, double *d_Y, double *d_R, void *d_scratch, void *stream);

/* Truncated Householder QR with column pivoting of count k x k matrices:
 * rank r = first step whose trailing Frobenius norm is <= tol; d_X (count x
 * k x k) receives Q1 in its first r columns, d_B (count x k x k) receives
 * B^T (k x r) with A ~ Q1 B.  d_rank: count int32.  d_scratch: at least
 * 512 + count * (8*k*k + 144) bytes.  Synchronises `stream`. */
tlr_status tlr_diag_qrcp(int32_t count, int32_t k, const double *d_A, double tol, double *d_X, double *d_B,
                         int32_t *d_rank, void *d_scratch, void *stream);

/* Singular values (descending) and left singular vectors of k x k matrices
 * by the one-sided Jacobi kernel of the compression step.  d_A: count
 * matrices, each k x k column-major, consecutive; d_S: count x k; d_X:
 * count x k x k.  d_rank: count int32, #{s > tol}.  k <= 512. */
tlr_status tlr_diag_svd(int32_t count, int32_t k, const double *d_A, double tol, double *d_S, double *d_X,
                        int32_t *d_rank, void *d_scratch, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TLRMLE_H */
