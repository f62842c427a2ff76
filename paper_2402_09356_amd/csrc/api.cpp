// extern "C" entry points declared in include/tlrmle.h.
#include <cmath>
#include "kernels.h"
#include "ktimer.h"

namespace tlr {
tlr_status plan_create(tlr_plan *out, int64_t n, int nb, int maxrank, tlr_precision prec, uint32_t flags);
void plan_destroy(tlr_plan p);
size_t plan_ws_bytes(tlr_plan p);
size_t plan_ws_bytes_budget(tlr_plan p, int64_t rank_budget);
tlr_status gen_tiles(tlr_plan p, const double *d_locs, tlr_theta th, void *d_ws, size_t ws_bytes, hipStream_t s);
tlr_status gen_tiles_bivariate(tlr_plan p, const double *d_locs, const tlr_theta_biv &th, void *d_ws, size_t ws_bytes,
                               hipStream_t s);
tlr_status compress(tlr_plan p, double tol, void *d_ws, size_t ws_bytes, int32_t *d_ranks, hipStream_t s);
tlr_status potrf(tlr_plan p, void *d_ws, size_t ws_bytes, hipStream_t s);
tlr_status solve_logdet(tlr_plan p, const double *d_z, void *d_ws, size_t ws_bytes, double *d_out, hipStream_t s);
tlr_status status_read(tlr_plan p, const void *d_ws, tlr_devinfo *out, hipStream_t s);
void plan_shape(tlr_plan p, int64_t *n, int32_t *nb, int32_t *nt, int32_t *maxrank);
tlr_status tile_read(tlr_plan p, const void *d_ws, int i, int j, double *d_out, int32_t *h_rank, hipStream_t s);
tlr_status ranks_read(tlr_plan p, const void *d_ws, int which, int32_t *d_out, hipStream_t s);
tlr_status batch_plan_create(tlr_batch_plan *out, int count, const int64_t *n, const int32_t *nb, int maxrank,
                             tlr_precision prec, uint32_t flags);
void batch_plan_destroy(tlr_batch_plan bp);
tlr_status batch_status_read(tlr_batch_plan bp, const void *d_ws, int index, tlr_devinfo *out, hipStream_t s);
size_t batch_ws_bytes(tlr_batch_plan bp);
tlr_status loglik_batched(tlr_batch_plan bp, const double *const *locs, const double *const *z,
                          const tlr_theta *theta, double tol, void *d_ws, size_t ws_bytes, double *d_out,
                          int workers, hipStream_t s);
}  // namespace tlr

static inline hipStream_t as_stream(void *s) { return static_cast<hipStream_t>(s); }

extern "C" {

size_t tlr_reorder_ws_bytes(int64_t n, tlr_ordering kind) { return tlr::reorder_ws_bytes(n, kind); }

tlr_status tlr_reorder(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                       int32_t *d_perm, void *d_ws, size_t ws_bytes, void *stream) {
    return tlr::reorder(d_locs, n, kind, seed, flags, d_perm, d_ws, ws_bytes, as_stream(stream));
}

tlr_status tlr_reorder_noalloc(const double *d_locs, int64_t n, tlr_ordering kind, uint64_t seed, uint32_t flags,
                               int32_t *d_perm, void *stream) {
    return tlr::reorder_noalloc(d_locs, n, kind, seed, flags, d_perm, as_stream(stream));
}

int64_t tlr_reorder_noalloc_max_n(void) { return tlr::reorder_noalloc_max_n(); }

tlr_status tlr_apply_perm(const int32_t *d_perm, int64_t n, const double *d_locs, const double *d_z,
                          double *d_locs_out, double *d_z_out, int32_t dequantize, void *stream) {
    return tlr::apply_perm(d_perm, n, d_locs, d_z, d_locs_out, d_z_out, dequantize, as_stream(stream));
}

tlr_status tlr_plan_create(tlr_plan *out, int64_t n, int32_t nb, int32_t maxrank, tlr_precision precision,
                           uint32_t flags) {
    return tlr::plan_create(out, n, nb, maxrank, precision, flags);
}

void tlr_plan_destroy(tlr_plan plan) { tlr::plan_destroy(plan); }

size_t tlr_plan_ws_bytes(tlr_plan plan, int64_t rank_budget) { return tlr::plan_ws_bytes_budget(plan, rank_budget); }

void tlr_plan_shape(tlr_plan plan, int64_t *n, int32_t *nb, int32_t *nt, int32_t *maxrank) {
    tlr::plan_shape(plan, n, nb, nt, maxrank);
}

tlr_status tlr_gen_tiles(tlr_plan plan, const double *d_locs, tlr_theta theta, void *d_ws, size_t ws_bytes,
                         void *stream) {
    return tlr::gen_tiles(plan, d_locs, theta, d_ws, ws_bytes, as_stream(stream));
}

tlr_status tlr_compress(tlr_plan plan, double tol, void *d_ws, size_t ws_bytes, int32_t *d_ranks, void *stream) {
    return tlr::compress(plan, tol, d_ws, ws_bytes, d_ranks, as_stream(stream));
}

tlr_status tlr_potrf(tlr_plan plan, void *d_ws, size_t ws_bytes, void *stream) {
    return tlr::potrf(plan, d_ws, ws_bytes, as_stream(stream));
}

tlr_status tlr_solve_logdet(tlr_plan plan, const double *d_z, void *d_ws, size_t ws_bytes, double *d_out,
                            void *stream) {
    return tlr::solve_logdet(plan, d_z, d_ws, ws_bytes, d_out, as_stream(stream));
}

tlr_status tlr_batch_plan_create(tlr_batch_plan *out, int32_t count, const int64_t *h_n, const int32_t *h_nb,
                                 int32_t maxrank, tlr_precision precision, uint32_t flags) {
    return tlr::batch_plan_create(out, count, h_n, h_nb, maxrank, precision, flags);
}

void tlr_batch_plan_destroy(tlr_batch_plan bplan) { tlr::batch_plan_destroy(bplan); }

size_t tlr_batch_ws_bytes(tlr_batch_plan bplan) { return tlr::batch_ws_bytes(bplan); }

tlr_status tlr_batch_status_read(tlr_batch_plan bplan, const void *d_ws, int32_t index, tlr_devinfo *out,
                                 void *stream) {
    return tlr::batch_status_read(bplan, d_ws, index, out, as_stream(stream));
}

tlr_status tlr_loglik_batched(tlr_batch_plan bplan, const double *const *h_locs, const double *const *h_z,
                              const tlr_theta *h_theta, double tol, void *d_ws, size_t ws_bytes, double *d_out,
                              int32_t workers, void *stream) {
    return tlr::loglik_batched(bplan, h_locs, h_z, h_theta, tol, d_ws, ws_bytes, d_out, workers, as_stream(stream));
}

tlr_status tlr_loglik(tlr_plan plan, const double *d_locs, const double *d_z, tlr_theta theta, double tol,
                      void *d_ws, size_t ws_bytes, double *d_out, int32_t *d_ranks, void *stream) {
    hipStream_t s = as_stream(stream);
    if (!plan || !d_locs || !d_z || !d_ws || !d_out) return TLR_E_INVAL;
    tlr_status st = tlr::gen_tiles(plan, d_locs, theta, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    st = tlr::compress(plan, tol, d_ws, ws_bytes, d_ranks, s);
    if (st != TLR_OK) return st;
    st = tlr::potrf(plan, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    return tlr::solve_logdet(plan, d_z, d_ws, ws_bytes, d_out, s);
}

tlr_status tlr_gen_tiles_bivariate(tlr_plan plan, const double *d_locs, tlr_theta_biv theta, void *d_ws,
                                   size_t ws_bytes, void *stream) {
    return tlr::gen_tiles_bivariate(plan, d_locs, theta, d_ws, ws_bytes, as_stream(stream));
}

tlr_status tlr_loglik_bivariate(tlr_plan plan, const double *d_locs, const double *d_z, tlr_theta_biv theta,
                                double tol, void *d_ws, size_t ws_bytes, double *d_out, int32_t *d_ranks,
                                void *stream) {
    hipStream_t s = as_stream(stream);
    if (!plan || !d_locs || !d_z || !d_ws || !d_out) return TLR_E_INVAL;
    tlr_status st = tlr::gen_tiles_bivariate(plan, d_locs, theta, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    st = tlr::compress(plan, tol, d_ws, ws_bytes, d_ranks, s);
    if (st != TLR_OK) return st;
    st = tlr::potrf(plan, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    return tlr::solve_logdet(plan, d_z, d_ws, ws_bytes, d_out, s);
}

static bool tgh_valid(const tlr_tgh &p) {
    return std::isfinite(p.xi) && std::isfinite(p.g) && std::isfinite(p.omega) && p.omega > 0.0 &&
           std::isfinite(p.h) && p.h >= 0.0;
}

tlr_status tlr_tgh_inverse(const double *d_t, int64_t n, tlr_tgh p, double *d_z, void *stream) {
    if (n < 0 || !tgh_valid(p) || (n > 0 && (!d_t || !d_z))) return TLR_E_INVAL;
    return tlr::tgh_inverse(d_t, n, p.xi, p.omega, p.g, p.h, d_z, as_stream(stream));
}

tlr_status tlr_loglik_tgh(tlr_plan plan, const double *d_locs, const double *d_t, tlr_theta theta, tlr_tgh p,
                          double tol, void *d_ws, size_t ws_bytes, double *d_z, double *d_out, void *stream) {
    hipStream_t s = as_stream(stream);
    if (!plan || !d_locs || !d_t || !d_z || !d_ws || !d_out || !tgh_valid(p)) return TLR_E_INVAL;
    int64_t n = 0;
    int32_t nb = 0, nt = 0, maxrank = 0;
    tlr::plan_shape(plan, &n, &nb, &nt, &maxrank);
    // generation first: it checks theta and the workspace before any launch
    tlr_status st = tlr::gen_tiles(plan, d_locs, theta, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    st = tlr::tgh_inverse(d_t, n, p.xi, p.omega, p.g, p.h, d_z, s);
    if (st != TLR_OK) return st;
    st = tlr::compress(plan, tol, d_ws, ws_bytes, nullptr, s);
    if (st != TLR_OK) return st;
    st = tlr::potrf(plan, d_ws, ws_bytes, s);
    if (st != TLR_OK) return st;
    st = tlr::solve_logdet(plan, d_z, d_ws, ws_bytes, d_out, s);
    if (st != TLR_OK) return st;
    return tlr::tgh_combine(d_z, n, p.omega, p.g, p.h, d_out, s);
}

tlr_status tlr_status_read(tlr_plan plan, const void *d_ws, tlr_devinfo *out, void *stream) {
    return tlr::status_read(plan, d_ws, out, as_stream(stream));
}

const char *tlr_strerror(tlr_status code) {
    switch (code) {
        case TLR_OK: return "ok";
        case TLR_E_INVAL: return "invalid argument";
        case TLR_E_NOMEM: return "workspace too small";
        case TLR_E_UNSUPPORTED: return "unsupported";
        case TLR_E_HIP: return "HIP runtime error";
        case TLR_NOT_SPD: return "matrix not positive definite";
        case TLR_RANK_OVERFLOW: return "tile rank above the rank cap";
        case TLR_E_DOMAIN: return "location outside the unit square";
        case TLR_ARENA_OVERFLOW: return "factor arena full (rank budget too small)";
        default: return "unknown status";
    }
}

const char *tlr_version(void) { return "tlrmle 0.1 (gfx950)"; }

tlr_status tlr_kstats_enable(int32_t on) {
    tlr::ktimer_enable(on != 0);
    return TLR_OK;
}

tlr_status tlr_kstats_select(const char *name) {
    tlr::ktimer_select((name && name[0]) ? tlr::ktimer_class(name) : -1);
    return TLR_OK;
}

tlr_status tlr_kstats_reset(void) {
    tlr::ktimer_reset();
    return TLR_OK;
}

int32_t tlr_kstats_read(tlr_kstat *out, int32_t max) {
    if (max > 0 && !out) return -1;
    static_assert(sizeof(tlr_kstat) == sizeof(tlr::KStat), "tlr_kstat layout");
    return tlr::ktimer_read(reinterpret_cast<tlr::KStat *>(out), max < 0 ? 0 : max);
}

tlr_status tlr_ranks_read(tlr_plan plan, const void *d_ws, int32_t which, int32_t *d_out, void *stream) {
    return tlr::ranks_read(plan, d_ws, which, d_out, as_stream(stream));
}

tlr_status tlr_diag_tile(tlr_plan plan, const void *d_ws, int32_t i, int32_t j, double *d_out, int32_t *h_rank,
                         void *stream) {
    return tlr::tile_read(plan, d_ws, i, j, d_out, h_rank, as_stream(stream));
}

}  // extern "C"

// ---------------------------------------------------------- diagnostics --
#include <vector>

static_assert(sizeof(tlr::SmallDesc) <= 128, "diag_svd scratch formula assumes <= 128-byte descriptors");

extern "C" tlr_status tlr_diag_gemm(int32_t trans_a, int32_t trans_b, int32_t M, int32_t N, int32_t K, double alpha,
                                    const double *d_A, int32_t lda, const double *d_B, int32_t ldb, double beta,
                                    double *d_C, int32_t ldc, void *stream) {
    if (M < 0 || N < 0 || K < 0 || !d_C || (K > 0 && (!d_A || !d_B))) return TLR_E_INVAL;
    if (M == 0 || N == 0) return TLR_OK;
    if (ldc < M || lda < (trans_a ? K : M) || ldb < (trans_b ? N : K)) return TLR_E_INVAL;
    hipStream_t s = as_stream(stream);
    tlr::GemmDesc g{};
    g.A = d_A;
    g.B = d_B;
    g.C = d_C;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = lda > 0 ? lda : 1;
    g.ldb = ldb > 0 ? ldb : 1;
    g.ldc = ldc;
    g.alpha = alpha;
    g.beta = beta;
    tlr::GemmDesc *d = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&d), sizeof(g), s) != hipSuccess) return TLR_E_HIP;
    tlr_status st = TLR_OK;
    if (hipMemcpyAsync(d, &g, sizeof(g), hipMemcpyHostToDevice, s) != hipSuccess) st = TLR_E_HIP;
    if (st == TLR_OK) st = tlr::gemm_batched(trans_a != 0, trans_b != 0, d, 1, M, N, s, &g);
    if (hipStreamSynchronize(s) != hipSuccess) st = TLR_E_HIP;
    (void)hipFreeAsync(d, s);
    (void)hipStreamSynchronize(s);
    return st;
}

extern "C" tlr_status tlr_diag_gemm_strided(int32_t trans_a, int32_t trans_b, int32_t count, int32_t M, int32_t N,
                                            int32_t K, double alpha, const double *d_A, int32_t lda, int64_t stride_a,
                                            const double *d_B, int32_t ldb, int64_t stride_b, double beta,
                                            double *d_C, int32_t ldc, int64_t stride_c, void *stream) {
    if (count < 0 || count > 65535 || M < 0 || N < 0 || K < 0 || !d_C || (K > 0 && (!d_A || !d_B)))
        return TLR_E_INVAL;
    if (count == 0 || M == 0 || N == 0) return TLR_OK;
    if (ldc < M || lda < (trans_a ? K : M) || ldb < (trans_b ? N : K)) return TLR_E_INVAL;
    if (stride_a < 0 || stride_b < 0 || stride_c < (int64_t)ldc * N) return TLR_E_INVAL;
    hipStream_t s = as_stream(stream);
    std::vector<tlr::GemmDesc> h(count);
    for (int t = 0; t < count; ++t) {
        tlr::GemmDesc g{};
        g.A = d_A + stride_a * t;
        g.B = d_B + stride_b * t;
        g.C = d_C + stride_c * t;
        g.M = M;
        g.N = N;
        g.K = K;
        g.lda = lda > 0 ? lda : 1;
        g.ldb = ldb > 0 ? ldb : 1;
        g.ldc = ldc;
        g.alpha = alpha;
        g.beta = beta;
        h[t] = g;
    }
    tlr::GemmDesc *d = nullptr;
    if (hipMallocAsync(reinterpret_cast<void **>(&d), sizeof(tlr::GemmDesc) * count, s) != hipSuccess)
        return TLR_E_HIP;
    tlr_status st = TLR_OK;
    if (hipMemcpyAsync(d, h.data(), sizeof(tlr::GemmDesc) * count, hipMemcpyHostToDevice, s) != hipSuccess)
        st = TLR_E_HIP;
    if (st == TLR_OK) st = tlr::gemm_batched(trans_a != 0, trans_b != 0, d, count, M, N, s, h.data());
    if (hipStreamSynchronize(s) != hipSuccess) st = TLR_E_HIP;
    (void)hipFreeAsync(d, s);
    (void)hipStreamSynchronize(s);
    return st;
}

extern "C" tlr_status tlr_diag_peak_hbm(const void *d_src, void *d_dst, int64_t bytes, int32_t reps,
                                        double *h_gbs, void *stream) {
    return tlr::peak_hbm(d_src, d_dst, bytes, reps, h_gbs, as_stream(stream));
}

extern "C" tlr_status tlr_diag_alloc_counts(int64_t *h_pinned, int64_t *h_streams) {
    if (!h_pinned || !h_streams) return TLR_E_INVAL;
    tlr::alloc_counts(h_pinned, h_streams);
    return TLR_OK;
}

extern "C" tlr_status tlr_diag_peak_mfma_f64(double *d_scratch, int64_t scratch_words, int32_t iters,
                                             double *h_tflops, void *stream) {
    return tlr::peak_mfma_f64(d_scratch, scratch_words, iters, h_tflops, as_stream(stream));
}

extern "C" tlr_status tlr_diag_svd(int32_t count, int32_t k, const double *d_A, double tol, double *d_S,
                                   double *d_X, int32_t *d_rank, void *d_scratch, void *stream) {
    if (count < 0 || k < 1 || k > tlr::kMaxSketch || !d_A || !d_S || !d_X || !d_rank || !d_scratch)
        return TLR_E_INVAL;
    if (count == 0) return TLR_OK;
    hipStream_t s = as_stream(stream);
    // d_scratch: count * (k*k doubles + 4 int32) + sizeof(DevParams) + descriptors
    char *w = static_cast<char *>(d_scratch);
    tlr::DevParams *params = reinterpret_cast<tlr::DevParams *>(w);
    w += 256;
    double *R = reinterpret_cast<double *>(w);
    w += sizeof(double) * (size_t)count * k * k;
    int32_t *stat = reinterpret_cast<int32_t *>(w);
    w += tlr::align_up(sizeof(int32_t) * 4 * (size_t)count, 256);
    tlr::SmallDesc *dd = reinterpret_cast<tlr::SmallDesc *>(w);
    std::vector<tlr::SmallDesc> h(count);
    for (int t = 0; t < count; ++t) {
        tlr::SmallDesc d{};
        d.A = const_cast<double *>(d_A) + (size_t)t * k * k;
        d.lda = k;
        d.R = R + (size_t)t * k * k;
        d.ldr = k;
        d.X = d_X + (size_t)t * k * k;
        d.ldx = k;
        d.S = d_S + (size_t)t * k;
        d.rank = stat + 4 * t;
        d.flag = stat + 4 * t + 2;
        d.k = k;
        d.k_full = k;
        h[t] = d;
    }
    if (hipMemsetAsync(params, 0, sizeof(tlr::DevParams), s) != hipSuccess) return TLR_E_HIP;
    if (hipMemcpyAsync(dd, h.data(), sizeof(tlr::SmallDesc) * count, hipMemcpyHostToDevice, s) != hipSuccess)
        return TLR_E_HIP;
    tlr_status st = tlr::jacobi_svd(dd, count, k, tol, 0, k, k, params, s);
    if (st != TLR_OK) return st;
    std::vector<int32_t> hs(4 * (size_t)count), hr(count);
    if (hipMemcpyAsync(hs.data(), stat, sizeof(int32_t) * 4 * count, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TLR_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return TLR_E_HIP;
    for (int t = 0; t < count; ++t) hr[t] = hs[4 * t + 1];
    if (hipMemcpy(d_rank, hr.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice) != hipSuccess) return TLR_E_HIP;
    return TLR_OK;
}

extern "C" tlr_status tlr_diag_qrcp(int32_t count, int32_t k, const double *d_A, double tol, double *d_X, double *d_B,
                                    int32_t *d_rank, void *d_scratch, void *stream) {
    if (count < 0 || k < 1 || k > tlr::kMaxSketch || !d_A || !d_X || !d_B || !d_rank || !d_scratch || !(tol >= 0.0))
        return TLR_E_INVAL;
    if (count == 0) return TLR_OK;
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(d_scratch);
    tlr::DevParams *params = reinterpret_cast<tlr::DevParams *>(w);
    w += 256;
    double *R = reinterpret_cast<double *>(w);
    w += sizeof(double) * (size_t)count * k * k;
    int32_t *stat = reinterpret_cast<int32_t *>(w);
    w += tlr::align_up(sizeof(int32_t) * 4 * (size_t)count, 256);
    tlr::SmallDesc *dd = reinterpret_cast<tlr::SmallDesc *>(w);
    std::vector<tlr::SmallDesc> h(count);
    for (int t = 0; t < count; ++t) {
        tlr::SmallDesc d{};
        d.A = const_cast<double *>(d_A) + (size_t)t * k * k;
        d.lda = k;
        d.R = R + (size_t)t * k * k;
        d.ldr = k;
        d.X = d_X + (size_t)t * k * k;
        d.ldx = k;
        d.Y = d_B + (size_t)t * k * k;
        d.ldy = k;
        d.rank = stat + 4 * t;
        d.flag = stat + 4 * t + 2;
        d.k = k;
        d.k_full = k;
        h[t] = d;
    }
    if (hipMemsetAsync(params, 0, sizeof(tlr::DevParams), s) != hipSuccess) return TLR_E_HIP;
    if (hipMemcpyAsync(dd, h.data(), sizeof(tlr::SmallDesc) * count, hipMemcpyHostToDevice, s) != hipSuccess)
        return TLR_E_HIP;
    tlr_status st = tlr::qrcp_trunc(dd, count, k, tol, 0, k, k, params, s);
    if (st != TLR_OK) return st;
    std::vector<int32_t> hs(4 * (size_t)count), hr(count);
    if (hipMemcpyAsync(hs.data(), stat, sizeof(int32_t) * 4 * count, hipMemcpyDeviceToHost, s) != hipSuccess)
        return TLR_E_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return TLR_E_HIP;
    for (int t = 0; t < count; ++t) hr[t] = hs[4 * t];
    if (hipMemcpy(d_rank, hr.data(), sizeof(int32_t) * count, hipMemcpyHostToDevice) != hipSuccess) return TLR_E_HIP;
    return TLR_OK;
}

extern "C" tlr_status tlr_diag_cholqr(int32_t m, int32_t k, double *d_Y, double *d_R, void *d_scratch, void *stream) {
    if (m < 1 || k < 1 || k > tlr::kMaxSketch || !d_Y || !d_R || !d_scratch) return TLR_E_INVAL;
    hipStream_t s = as_stream(stream);
    char *w = static_cast<char *>(d_scratch);
    tlr::DevParams *params = reinterpret_cast<tlr::DevParams *>(w);
    w += 256;
    double *G = reinterpret_cast<double *>(w);
    double *Rp[4], *T = G + (size_t)k * k;
    for (int q = 0; q < 4; ++q) Rp[q] = T + (size_t)(q + 1) * k * k;
    double *T2 = Rp[3] + (size_t)k * k;
    char *dsc = reinterpret_cast<char *>(T2 + (size_t)k * k);
    if (hipMemsetAsync(params, 0, sizeof(tlr::DevParams), s) != hipSuccess) return TLR_E_HIP;
    // descriptors: 4 Gram products, 4 small descs, 3 R products
    tlr::GemmDesc hg[8];
    tlr::SmallDesc hsd[4];
    for (int it = 0; it < 4; ++it) {
        tlr::GemmDesc g{};
        g.A = d_Y; g.B = d_Y; g.C = G; g.M = k; g.N = k; g.K = m; g.lda = m; g.ldb = m; g.ldc = k;
        g.alpha = 1.0; g.beta = 0.0;
        hg[it] = g;
        tlr::SmallDesc d{};
        d.A = G; d.lda = k; d.R = Rp[it]; d.ldr = k; d.X = T2; d.Y = d_Y; d.ldy = m; d.m = m; d.k = k;
        hsd[it] = d;
    }
    auto mul = [&](const double *A, const double *B, double *C) {
        tlr::GemmDesc g{};
        g.A = A; g.B = B; g.C = C; g.M = k; g.N = k; g.K = k; g.lda = k; g.ldb = k; g.ldc = k;
        g.alpha = 1.0; g.beta = 0.0;
        return g;
    };
    hg[4] = mul(Rp[3], Rp[2], T);
    hg[5] = mul(T, Rp[1], T2);
    hg[6] = mul(T2, Rp[0], d_R);
    tlr::GemmDesc *dg = reinterpret_cast<tlr::GemmDesc *>(dsc);
    tlr::SmallDesc *ds = reinterpret_cast<tlr::SmallDesc *>(dsc + tlr::align_up(sizeof(hg), 256));
    if (hipMemcpyAsync(dg, hg, sizeof(hg), hipMemcpyHostToDevice, s) != hipSuccess) return TLR_E_HIP;
    if (hipMemcpyAsync(ds, hsd, sizeof(hsd), hipMemcpyHostToDevice, s) != hipSuccess) return TLR_E_HIP;
    for (int it = 0; it < 4; ++it) {
        tlr_status st = tlr::gemm_batched(true, false, dg + it, 1, k, k, s);
        if (st == TLR_OK) st = tlr::chol_small(ds + it, 1, k, it < 2 ? 1 : 2, params, s);
        if (st == TLR_OK) st = tlr::trsm_rows(ds + it, 1, m, k, s);
        if (st != TLR_OK) return st;
    }
    for (int q = 4; q < 7; ++q) {
        tlr_status st = tlr::gemm_batched(false, false, dg + q, 1, k, k, s);
        if (st != TLR_OK) return st;
    }
    if (hipStreamSynchronize(s) != hipSuccess) return TLR_E_HIP;
    return TLR_OK;
}
