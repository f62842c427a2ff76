// Plan, workspace layout and the host-side drivers of the TLR likelihood:
// covariance generation, per-tile randomised compression, the left-looking
// TLR Cholesky factorisation and the forward solve.
//
// Workspace (caller-owned device memory, offsets fixed by the plan):
//   params    DevParams + Matern constants + hint marker
//   x, y      ordered coordinates, structure-of-arrays, padded to nt*nb
//   diag      nt dense nb x nb diagonal tiles (column-major)
//   rsig, rL  nt x nt int32 rank tables: compressed Sigma, current factor
//   tstat     per off-diagonal tile: {rank used, numerical rank, retry flag, -}
//   tofs      per off-diagonal tile (i > j, index i(i-1)/2 + j): offset and
//             width of its factor slot in the factor arena, then the arena's
//             fill mark
//   yvec      padded solve vector
//   omega     nb x kmax standard-normal test matrix of the range finder
//   desc      kernel descriptor staging area
//   arena     per-wave scratch (dense tiles, sketches, small matrices)
//   fac       factor arena, to the end of the caller's workspace: each tile's
//             U then V (nb x w, column-major, w >= its rank), placed by the
//             host as ranks become known (first fit at the fill mark; a
//             recompressed tile reuses its slot when the new rank fits)
#include <algorithm>
#include <atomic>
#include <functional>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <utility>
#include <vector>

#include "kernels.h"
#include "ktimer.h"

struct tlr_plan_s {
    int64_t n, npad, ntiles;
    int nb, nt, rcap, kmax, pover, min_tail, k0;
    tlr_precision prec;
    uint32_t flags;
    size_t off_params, off_x, off_y, off_diag, off_rsig, off_rL, off_tstat, off_tofs, off_yvec, off_omega,
        off_desc, off_arena, off_knu, off_dense, off_wide, off_nrm_s, off_nrm_l, off_noise, off_linv, off_ysol, off_fac;
    bool mixed;  // TLR_MIXED_FP32: low-rank factors stored in float32
    int fw;      // bytes per stored factor entry (8, or 4 when mixed)
    bool dense_ok;   // TLR_PLAN_DENSE_TILES: over-rank tiles kept dense in the wide slots
    bool svd_trunc;  // TLR_PLAN_SVD_TRUNCATION: truncate by singular values, not pivoted QR
    size_t desc_bytes, arena_bytes, ws_bytes;
};

namespace tlr {
namespace {

constexpr uint64_t kHintMagic = 0x544c524d4c453031ull;  // ranks in rsig are valid hints
constexpr uint64_t kSketchSeed = 0x5eed5ca1ab1e2024ull;
constexpr int kMaxWave = 4096;  // tile jobs per batched launch sequence

struct ParamsBlock {
    DevParams dp;
    MaternConst mc;
    BivConst bv;  // bv.on: the bivariate model's generator replaces mc's
    uint64_t hint_magic;
    double tol;
};

inline int64_t tile_index(int i, int j) { return (int64_t)i * (i - 1) / 2 + j; }

bool debug_enabled() {
    static const bool on = [] {
        const char *e = std::getenv("TLR_DEBUG");
        return e && *e && *e != '0';
    }();
    return on;
}

// Pinned host staging buffers for descriptor uploads (asynchronous DMA
// copies), kept for the life of the process.  A buffer goes back to the pool
// only after its stream has drained, so no copy from it is still in flight
// when another context takes it.
std::atomic<int64_t> g_pinned_allocs{0}, g_streams_created{0};

class PinnedPool {
  public:
    char *get(size_t bytes, size_t *cap) {
        {
            // the smallest free buffer that fits
            std::lock_guard<std::mutex> g(mu_);
            size_t best = free_.size();
            for (size_t i = 0; i < free_.size(); ++i)
                if (free_[i].second >= bytes && (best == free_.size() || free_[i].second < free_[best].second))
                    best = i;
            if (best < free_.size()) {
                auto b = free_[best];
                free_.erase(free_.begin() + (std::ptrdiff_t)best);
                *cap = b.second;
                return b.first;
            }
        }
        void *h = nullptr;
        if (hipHostMalloc(&h, bytes, hipHostMallocDefault) != hipSuccess) return nullptr;
        note_pinned_alloc();
        *cap = bytes;
        return static_cast<char *>(h);
    }
    void put(char *b, size_t cap) {
        std::lock_guard<std::mutex> g(mu_);
        free_.emplace_back(b, cap);
    }

  private:
    std::mutex mu_;
    std::vector<std::pair<char *, size_t>> free_;
};

// Side streams (default priority) with the two events that order work on
// them against a context's main stream; per device, kept for the life of the
// process and handed out to one context at a time.
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t from_main = nullptr, from_side = nullptr;
    int dev = -1;
};

class SidePool {
  public:
    bool get(SideStream *out) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return false;
        {
            std::lock_guard<std::mutex> g(mu_);
            for (size_t i = 0; i < free_.size(); ++i)
                if (free_[i].dev == dev) {
                    *out = free_[i];
                    free_.erase(free_.begin() + (std::ptrdiff_t)i);
                    return true;
                }
        }
        SideStream n;
        n.dev = dev;
        if (hipStreamCreateWithFlags(&n.s, hipStreamNonBlocking) != hipSuccess) return false;
        note_stream_created();
        if (hipEventCreateWithFlags(&n.from_main, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&n.from_side, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return false;  // leaked on this rare path; the context then stays on one stream
        }
        *out = n;
        return true;
    }
    void put(const SideStream &st) {
        std::lock_guard<std::mutex> g(mu_);
        free_.push_back(st);
    }

  private:
    std::mutex mu_;
    std::vector<SideStream> free_;
};

SidePool &side_pool() {
    static SidePool *pool = new SidePool();  // never destroyed
    return *pool;
}

PinnedPool &pinned_pool() {
    static PinnedPool *pool = new PinnedPool();  // never destroyed: outlives static teardown
    return *pool;
}

struct Ctx {
    const tlr_plan_s *p;
    char *ws;
    hipStream_t s;
    char *hdesc = nullptr;          // pinned staging (pageable fallback below)
    size_t hdesc_cap = 0;
    std::vector<char> hdesc_pageable;
    bool in_flight = false;         // uploads issued since the last stream sync
    size_t desc_used = 0;
    size_t flushed = 0;             // staged descriptor bytes already on the device
    size_t arena_used = 0;
    size_t arena_off = 0, arena_cap = 0;  // the scratch arena in use (the plan's, or a larger one)

    Ctx(const tlr_plan_s *plan, void *w, hipStream_t st)
        : p(plan), ws(static_cast<char *>(w)), s(st), arena_off(plan->off_arena), arena_cap(plan->arena_bytes) {
        hdesc = pinned_pool().get(plan->desc_bytes, &hdesc_cap);
        if (!hdesc) {
            hdesc_pageable.resize(plan->desc_bytes);
            hdesc = hdesc_pageable.data();
        }
    }
    ~Ctx() {
        if (in_flight) (void)hipStreamSynchronize(s);
        if (side.s) {
            (void)hipStreamSynchronize(side.s);
            side_pool().put(side);
        }
        if (hdesc_pageable.empty() && hdesc) pinned_pool().put(hdesc, hdesc_cap);
        if (hstat_pageable.empty() && hstat) pinned_pool().put(reinterpret_cast<char *>(hstat), hstat_cap);
    }
    // A second stream for work that may run beside the main stream's (the
    // dense Cholesky of a diagonal tile beside the recompression of the tiles
    // below it).  fork() makes it wait for everything issued on the main
    // stream so far; join() makes the main stream wait for everything issued
    // on it.  Staged descriptors stay valid until sync_reset(), which drains
    // both streams.  Without a side stream both calls are no-ops and the work
    // simply runs on the main stream.
    SideStream side;
    bool side_busy = false;
    hipStream_t fork() {
        if (!side.s && !side_pool().get(&side)) return s;
        if (hipEventRecord(side.from_main, s) != hipSuccess || hipStreamWaitEvent(side.s, side.from_main, 0) != hipSuccess)
            return s;
        side_busy = true;
        return side.s;
    }
    tlr_status join() {
        if (!side_busy) return TLR_OK;
        TLR_HIP(hipEventRecord(side.from_side, side.s));
        TLR_HIP(hipStreamWaitEvent(s, side.from_side, 0));
        return TLR_OK;
    }
    tlr_status drain_side() {
        if (side_busy) {
            TLR_HIP(hipStreamSynchronize(side.s));
            side_busy = false;
        }
        return TLR_OK;
    }
    Ctx(const Ctx &) = delete;
    Ctx &operator=(const Ctx &) = delete;
    DevParams *params() const { return reinterpret_cast<DevParams *>(ws + p->off_params); }
    ParamsBlock *pblock() const { return reinterpret_cast<ParamsBlock *>(ws + p->off_params); }
    double *x() const { return reinterpret_cast<double *>(ws + p->off_x); }
    double *y() const { return reinterpret_cast<double *>(ws + p->off_y); }
    double *diag(int k) const {
        return reinterpret_cast<double *>(ws + p->off_diag) + (int64_t)k * p->nb * p->nb;
    }
    int32_t *rsig() const { return reinterpret_cast<int32_t *>(ws + p->off_rsig); }
    int32_t *rL() const { return reinterpret_cast<int32_t *>(ws + p->off_rL); }
    int32_t *tstat(int64_t t) const { return reinterpret_cast<int32_t *>(ws + p->off_tstat) + 4 * t; }
    // per-tile dense flags (host copy; loaded by load_dense, kept in the workspace)
    std::vector<int32_t> dflag;
    bool dense(int i, int j) const { return !dflag.empty() && dflag[(size_t)i * p->nt + j] != 0; }
    int32_t *ddense() const { return reinterpret_cast<int32_t *>(ws + p->off_dense); }
    double *wideU(int i, int j) const {
        return reinterpret_cast<double *>(ws + p->off_wide) + tile_index(i, j) * 2 * (int64_t)p->nb * p->nb;
    }
    double *wideV(int i, int j) const { return wideU(i, j) + (int64_t)p->nb * p->nb; }
    // low-rank factors of tile (i, j): float64, or float32 in a mixed plan
    // (fac_types() gives the GEMM type bits of such an operand)
    // factor slots: host copy of the tile table (loaded by load_slots)
    struct Slot {
        int64_t off;  // first entry of U in the factor arena
        int32_t w;    // columns reserved for U and for V
        int32_t pad;
    };
    std::vector<Slot> slots;
    int64_t fac_fill = 0;    // entries of the arena in use
    size_t ws_size = 0;      // the caller's workspace bytes (bounds the arena)
    void *U(int i, int j) const {
        if (dense(i, j)) return wideU(i, j);
        const Slot &sl = slots[(size_t)tile_index(i, j)];
        return ws + p->off_fac + sl.off * p->fw;
    }
    void *V(int i, int j) const {
        if (dense(i, j)) return wideV(i, j);
        const Slot &sl = slots[(size_t)tile_index(i, j)];
        return ws + p->off_fac + (sl.off + (int64_t)p->nb * sl.w) * p->fw;
    }
    int64_t fac_capacity() const { return (int64_t)((ws_size - p->off_fac) / p->fw); }
    // A slot of width w for tile (i, j): the tile's own when it is wide
    // enough, else a new one at the fill mark.  False when the arena is full.
    bool take_slot(int i, int j, int w) {
        Slot &sl = slots[(size_t)tile_index(i, j)];
        if (w <= sl.w) return true;
        const int64_t need = 2 * (int64_t)p->nb * w;
        if (fac_fill + need > fac_capacity()) return false;
        sl.off = fac_fill;
        sl.w = w;
        fac_fill += need;
        return true;
    }
    // Scratch for a compression wave: the plan's arena, or the free tail of
    // the factor arena when that is larger (a workspace sized for maxrank
    // slots holds far more than the factors need).  A wave's new slots must
    // stay below the tail taken: a job's scratch holds at least the nb x nb
    // tile and four nb x k panels (8 (nb^2 + 4 nb k) bytes), its slot at most
    // 2 nb k entries of 8 bytes, so the slots of a wave need at most
    // rho = 2 k / (nb + 4 k) of its scratch, k <= kmax; a share
    // 1 / (1 + rho) of the free space (less 2%) leaves them room.
    void use_free_tail() {
        arena_off = p->off_arena;
        arena_cap = p->arena_bytes;
        const size_t fill_end = p->off_fac + (size_t)fac_fill * p->fw;
        if (ws_size <= fill_end + 4096) return;
        const double rho = 2.0 * p->kmax / ((double)p->nb + 4.0 * p->kmax);
        const size_t tail = (size_t)((double)(ws_size - fill_end) * 0.98 / (1.0 + rho)) & ~(size_t)255;
        if (tail <= arena_cap) return;
        arena_off = (ws_size - tail) & ~(size_t)255;
        arena_cap = tail;
    }
    void reset_slots() {
        slots.assign((size_t)std::max<int64_t>(p->ntiles, 1), Slot{0, 0, 0});
        fac_fill = 0;
    }
    tlr_status load_slots() {
        slots.resize((size_t)std::max<int64_t>(p->ntiles, 1) + 1);
        TLR_HIP(hipMemcpyAsync(slots.data(), ws + p->off_tofs, sizeof(Slot) * slots.size(), hipMemcpyDeviceToHost,
                               s));
        TLR_HIP(hipStreamSynchronize(s));
        fac_fill = slots.back().off;
        slots.pop_back();
        return TLR_OK;
    }
    tlr_status store_slots() {
        slots.push_back(Slot{fac_fill, 0, 0});
        TLR_HIP(hipMemcpyAsync(ws + p->off_tofs, slots.data(), sizeof(Slot) * slots.size(), hipMemcpyHostToDevice,
                               s));
        TLR_HIP(hipStreamSynchronize(s));  // the host table is edited again after this
        slots.pop_back();
        return TLR_OK;
    }
    // first failure wins: record a failure the host detected
    tlr_status host_fail(int code, int i, int j) {
        int32_t cur = 0;
        TLR_HIP(hipMemcpyAsync(&cur, &params()->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TLR_HIP(hipStreamSynchronize(s));
        if (cur != 0) return TLR_OK;
        const int32_t v[3] = {code, i, j};
        TLR_HIP(hipMemcpyAsync(&params()->status, v, 3 * sizeof(int32_t), hipMemcpyHostToDevice, s));
        TLR_HIP(hipStreamSynchronize(s));
        return TLR_OK;
    }
    int fa() const { return p->mixed ? kGemmA32 : 0; }   // factor as left operand
    int fb() const { return p->mixed ? kGemmB32 : 0; }   // factor as right operand
    int fc() const { return p->mixed ? kGemmC32 : 0; }   // factor as result
    double *nrm_s() const { return reinterpret_cast<double *>(ws + p->off_nrm_s); }
    double *nrm_l() const { return reinterpret_cast<double *>(ws + p->off_nrm_l); }
    double *noise(int64_t t) const { return reinterpret_cast<double *>(ws + p->off_noise) + t; }
    double *linv(int j) const { return reinterpret_cast<double *>(ws + p->off_linv) + (int64_t)j * p->nb * p->nb; }
    double *ysol() const { return reinterpret_cast<double *>(ws + p->off_ysol); }
    tlr_status load_dense() {
        dflag.assign((size_t)p->nt * p->nt, 0);
        TLR_HIP(hipMemcpyAsync(dflag.data(), ddense(), sizeof(int32_t) * dflag.size(), hipMemcpyDeviceToHost, s));
        TLR_HIP(hipStreamSynchronize(s));
        return TLR_OK;
    }
    tlr_status store_dense() {
        if (dflag.empty()) dflag.assign((size_t)p->nt * p->nt, 0);
        TLR_HIP(hipMemcpyAsync(ddense(), dflag.data(), sizeof(int32_t) * dflag.size(), hipMemcpyHostToDevice, s));
        in_flight = true;
        return TLR_OK;
    }
    double *yvec() const { return reinterpret_cast<double *>(ws + p->off_yvec); }
    double *omega() const { return reinterpret_cast<double *>(ws + p->off_omega); }

    // Stage a descriptor array; it reaches the device at the next flush()
    // (one copy for everything staged since the last one).  nullptr when full.
    template <class T>
    T *push(const T *data, size_t count) {
        const size_t bytes = align_up(sizeof(T) * std::max<size_t>(count, 1), 256);
        if (desc_used + bytes > p->desc_bytes) return nullptr;
        std::memcpy(hdesc + desc_used, data, sizeof(T) * count);
        T *d = reinterpret_cast<T *>(ws + p->off_desc + desc_used);
        desc_used += bytes;
        return d;
    }
    tlr_status flush() {
        if (desc_used > flushed) {
            TLR_HIP(hipMemcpyAsync(ws + p->off_desc + flushed, hdesc + flushed, desc_used - flushed,
                                   hipMemcpyHostToDevice, s));
            in_flight = true;
            flushed = desc_used;
        }
        return TLR_OK;
    }
    template <class T>
    T *push(const std::vector<T> &v) {
        return push(v.data(), v.size());
    }
    // a panel of `elems` factor entries (float64, or float32 in a mixed plan)
    void *alloc_fac(size_t elems) { return alloc((elems * p->fw + 7) / 8); }
    void *fac_at(const void *base, size_t elems) const {
        return const_cast<char *>(static_cast<const char *>(base)) + elems * p->fw;
    }
    double *alloc(size_t words) {
        const size_t bytes = align_up(std::max<size_t>(words, 1) * sizeof(double), 256);
        if (arena_used + bytes > arena_cap) return nullptr;
        double *d = reinterpret_cast<double *>(ws + arena_off + arena_used);
        arena_used += bytes;
        return d;
    }
    // Wait for the main stream only (the side stream keeps running); staged
    // descriptors stay where they are, since the side stream may still read
    // some of them.
    tlr_status sync_main() {
        TLR_HIP(hipStreamSynchronize(s));
        in_flight = false;
        ktimer_poll();
        return TLR_OK;
    }
    tlr_status sync_reset() {
        TLR_HIP(hipStreamSynchronize(s));
        TLR_TRY(drain_side());
        in_flight = false;
        ktimer_poll();
        desc_used = 0;
        flushed = 0;
        return TLR_OK;
    }
    // The four status words of every job of a wave, with one copy of the
    // tile range they span, into pinned memory (so that both copies queue
    // behind the wave's kernels without holding the host); valid after the
    // next stream synchronisation and until the next read_stats.
    struct StatRead {
        const int32_t *raw = nullptr;
        int64_t t0 = 0;
        const int32_t *status = nullptr;  // the device status word, read in the same copy batch
    };
    int32_t *hstat = nullptr;  // pinned landing area of read_stats (pageable fallback below)
    size_t hstat_cap = 0;
    std::vector<int32_t> hstat_pageable;
    template <class JobT>
    tlr_status read_stats(const std::vector<JobT> &jobs, StatRead &sr) {
        if (jobs.empty()) return TLR_OK;
        int64_t lo = INT64_MAX, hi = -1;
        for (const auto &jb : jobs) {
            const int64_t t = tile_index(jb.i, jb.j);
            lo = std::min(lo, t);
            hi = std::max(hi, t);
        }
        if (!hstat) {
            // every tile's words and the status word: enough for any wave
            const size_t bytes = sizeof(int32_t) * (4 * (size_t)std::max<int64_t>(p->ntiles, 1) + 1);
            hstat = reinterpret_cast<int32_t *>(pinned_pool().get(bytes, &hstat_cap));
            if (!hstat) {
                hstat_pageable.resize(bytes / sizeof(int32_t));
                hstat = hstat_pageable.data();
            }
        }
        const size_t words = (size_t)(hi - lo + 1) * 4;
        sr.t0 = lo;
        sr.raw = hstat;
        sr.status = hstat + words;
        TLR_HIP(hipMemcpyAsync(hstat, tstat(lo), sizeof(int32_t) * words, hipMemcpyDeviceToHost, s));
        TLR_HIP(hipMemcpyAsync(hstat + words, &params()->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        in_flight = true;  // the copies land in pooled memory: wait before handing it back
        return TLR_OK;
    }
    tlr_status read_status(int *code) {
        int32_t st = 0;
        TLR_TRY(join());
        TLR_HIP(hipMemcpyAsync(&st, &params()->status, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        TLR_HIP(hipStreamSynchronize(s));
        TLR_TRY(drain_side());
        *code = st;
        return TLR_OK;
    }
};

// Launch a kernel wrapper after the staged descriptors reach the device.
#define TLR_LAUNCH(ctx, call)     \
    do {                          \
        TLR_TRY((ctx).flush());   \
        TLR_TRY(call);            \
    } while (0)

#define TLR_PUSH(ptr, ctx, vec)                          \
    auto ptr = (ctx).push(vec);                          \
    do {                                                 \
        if (!(ptr)) return TLR_E_NOMEM;                  \
    } while (0)

GemmDesc gd(const void *A, int lda, const void *B, int ldb, void *C, int ldc, int M, int N, int K,
            double alpha, double beta) {
    GemmDesc g{};
    g.A = A;
    g.B = B;
    g.C = C;
    g.M = M;
    g.N = N;
    g.K = K;
    g.lda = std::max(lda, 1);
    g.ldb = std::max(ldb, 1);
    g.ldc = std::max(ldc, 1);
    g.alpha = alpha;
    g.beta = beta;
    return g;
}

tlr_status launch_gemms(Ctx &c, bool ta, bool tb, const std::vector<GemmDesc> &v, int types = 0) {
    if (v.empty()) return TLR_OK;
    int mm = 0, mn = 0;
    for (const auto &g : v) {
        mm = std::max(mm, g.M_dev ? c.p->kmax : g.M);
        mn = std::max(mn, g.N_dev ? c.p->rcap : g.N);
    }
    if (mm <= 0 || mn <= 0) return TLR_OK;
    for (size_t off = 0; off < v.size(); off += 65535) {
        const size_t cnt = std::min<size_t>(65535, v.size() - off);
        auto *d = c.push(v.data() + off, cnt);
        if (!d) return TLR_E_NOMEM;
        TLR_LAUNCH(c, gemm_batched(ta, tb, d, (int)cnt, mm, mn, c.s, v.data() + off, false, types));
    }
    return TLR_OK;
}

// A GEMM batch staged in the descriptor area, launched later: staging every
// batch of a sequence first lets one upload carry all their descriptors.
struct StagedGemm {
    const GemmDesc *d = nullptr;
    const GemmDesc *h = nullptr;
    int count = 0, mm = 0, mn = 0;
    bool ta = false, tb = false;
    bool lower = false;  // only the lower triangle of each product is needed
    int types = 0;       // float32 operands (kGemm*32 bits)
};

tlr_status stage_gemms(Ctx &c, bool ta, bool tb, const std::vector<GemmDesc> &v, StagedGemm *out,
                       bool lower = false, int types = 0) {
    *out = StagedGemm{};
    if (v.empty()) return TLR_OK;
    if (v.size() > 65535) return TLR_E_UNSUPPORTED;
    int mm = 0, mn = 0;
    for (const auto &g : v) {
        mm = std::max(mm, g.M_dev ? c.p->kmax : g.M);
        mn = std::max(mn, g.N_dev ? c.p->rcap : g.N);
    }
    auto *d = c.push(v.data(), v.size());
    if (!d) return TLR_E_NOMEM;
    *out = StagedGemm{d, v.data(), (int)v.size(), mm, mn, ta, tb, lower, types};
    return TLR_OK;
}

tlr_status launch_staged(Ctx &c, const StagedGemm &g) {
    if (g.count == 0 || g.mm <= 0 || g.mn <= 0) return TLR_OK;
    TLR_LAUNCH(c, gemm_batched(g.ta, g.tb, g.d, g.count, g.mm, g.mn, c.s, g.h, g.lower, g.types));
    return TLR_OK;
}

// One tile compression problem for the randomised range finder.
struct Job {
    int i, j, k, kfull;
    // operator: dense tile A, or the Schur form U V^T - Xi Yj^T
    const double *A = nullptr;
    const void *Uop = nullptr, *Vop = nullptr;  // stored factors (float32 in a mixed plan)
    int r = 0;
    const void *Xi = nullptr;  // Schur panel X_i (factor element type)
    // outputs
    void *Uout = nullptr, *Vout = nullptr;
    const double *noise = nullptr;  // rounding-noise norm of the operator (mixed plans)
    int32_t *stat = nullptr;
    // buffers
    double *Yb = nullptr, *Zb = nullptr, *G = nullptr, *T = nullptr, *Rt = nullptr, *Xs = nullptr, *S = nullptr,
           *P = nullptr, *H = nullptr, *F = nullptr;
    double *D = nullptr;  // nb x nb: explicit Schur complement of a tile kept dense
    double *Rp[4] = {nullptr, nullptr, nullptr, nullptr};
};

size_t job_words(int nb, int k, int r, int R, bool dense) {
    size_t w = 0;
    if (dense) w += (size_t)nb * nb;
    w += 2 * (size_t)nb * k;          // Yb, Zb
    w += 9 * (size_t)k * k;           // G R1..R4 T Rt Xs P
    w += (size_t)k;                   // S
    w += (size_t)std::max(r, 1) * k;  // H
    w += (size_t)std::max(R, 1) * k;  // F
    w += 2 * (size_t)nb * k;          // U, V results (width k >= rank) before they go to their slot
    return w + 16 * 64;               // alignment slack
}

bool alloc_job(Ctx &c, Job &jb, int R) {
    const int nb = c.p->nb, k = jb.k;
    jb.Yb = c.alloc((size_t)nb * k);
    jb.Zb = c.alloc((size_t)nb * k);
    jb.G = c.alloc((size_t)k * k);
    for (int q = 0; q < 4; ++q) jb.Rp[q] = c.alloc((size_t)k * k);
    jb.T = c.alloc((size_t)k * k);
    jb.Rt = c.alloc((size_t)k * k);
    jb.Xs = c.alloc((size_t)k * k);
    jb.P = c.alloc((size_t)k * k);
    jb.S = c.alloc((size_t)k);
    jb.H = c.alloc((size_t)std::max(jb.r, 1) * k);
    jb.F = c.alloc((size_t)std::max(R, 1) * k);
    return jb.Yb && jb.Zb && jb.G && jb.Rp[0] && jb.Rp[1] && jb.Rp[2] && jb.Rp[3] && jb.T && jb.Rt && jb.Xs &&
           jb.P && jb.S && jb.H && jb.F;
}

// out_t = op_t(in_t) (trans: op^T).  in_t == nullptr means the test matrix.
// Staged first (descriptors in the descriptor area, host copies owned by
// the StagedApply, which must stay where it is until launched), launched
// later: staging every product and CholeskyQR of a range finder before its
// first launch lets one upload carry all their descriptors.
struct StagedApply {
    std::vector<GemmDesc> g1, g2, g3;  // factors and Schur panels share one element type
    StagedGemm s1, s2, s3;
};

tlr_status stage_apply(Ctx &c, std::vector<Job> &jobs, bool trans, bool from_omega, bool into_z, const void *Yj,
                       int Rj, StagedApply &a) {
    const int nb = c.p->nb;
    std::vector<GemmDesc> &g1 = a.g1, &g2 = a.g2, &g3 = a.g3;
    const bool dense = jobs.front().A != nullptr;
    // Yj^T W is the same for every job of the column (W is one matrix, a job
    // of width k reads its first k columns): form it once, at the widest
    // job's width, in that job's F, and let every job read its prefix.
    const Job *shared_f = nullptr;
    if (!dense && from_omega && !trans) {
        shared_f = &jobs.front();
        for (auto &jb : jobs)
            if (jb.k > shared_f->k) shared_f = &jb;
        g1.push_back(gd(Yj, nb, c.omega(), nb, shared_f->F, std::max(Rj, 1), Rj, shared_f->k, nb, 1.0, 0.0));
    }
    for (auto &jb : jobs) {
        const double *in = from_omega ? c.omega() : (into_z ? jb.Yb : jb.Zb);
        double *out = into_z ? jb.Zb : jb.Yb;
        if (dense) {
            g1.push_back(gd(jb.A, nb, in, nb, out, nb, nb, jb.k, nb, 1.0, 0.0));
        } else {
            // H = (trans ? U : V)^T in ; F = (trans ? Xi : Yj)^T in
            const void *left = trans ? jb.Uop : jb.Vop;
            const void *big = trans ? jb.Xi : Yj;
            double *F = shared_f ? shared_f->F : jb.F;
            g1.push_back(gd(left, nb, in, nb, jb.H, std::max(jb.r, 1), jb.r, jb.k, nb, 1.0, 0.0));
            if (!shared_f) g1.push_back(gd(big, nb, in, nb, F, std::max(Rj, 1), Rj, jb.k, nb, 1.0, 0.0));
            // out = (trans ? V : U) H ; out -= (trans ? Yj : Xi) F
            const void *right = trans ? jb.Vop : jb.Uop;
            const void *big2 = trans ? Yj : jb.Xi;
            g2.push_back(gd(right, nb, jb.H, std::max(jb.r, 1), out, nb, nb, jb.k, jb.r, 1.0, 0.0));
            g3.push_back(gd(big2, nb, F, std::max(Rj, 1), out, nb, nb, jb.k, Rj, -1.0, 1.0));
        }
    }
    if (dense) return stage_gemms(c, trans, false, g1, &a.s1);
    TLR_TRY(stage_gemms(c, true, false, g1, &a.s1, false, c.fa()));
    TLR_TRY(stage_gemms(c, false, false, g2, &a.s2, false, c.fa()));
    return stage_gemms(c, false, false, g3, &a.s3, false, c.fa());
}

tlr_status launch_apply(Ctx &c, const StagedApply &a) {
    TLR_TRY(launch_staged(c, a.s1));
    TLR_TRY(launch_staged(c, a.s2));
    return launch_staged(c, a.s3);
}

// CholeskyQR of each job's panel (nb x k) in place, four passes: two with
// the stabilising shift of shifted CholeskyQR (Fukaya et al. 2020) -- the
// panels are rank-deficient by construction (sketch width above the rank)
// and each shifted pass lifts the directions it cannot resolve yet -- then two
// plain passes with deflation of null directions, which restore
// orthonormality to rounding level.  Optionally R = R4 R3 R2 R1 (panel = Q R).
// With passes = 2 or 3 the result spans the panel's range with every
// direction above the rounding level lifted to unit size, which is all the
// first basis of the range finder needs.  With `shifted` = 1 and passes = 3
// (one shifted pass, two deflating ones) the directions above about 1e-11 of
// the panel's norm come out orthonormal and the rest are deflated: enough when
// the truncation threshold lies above that (see full_passes).  Staged and
// launched in two halves like the products above; staging moves each job's
// Rt to where the launched passes leave it.
struct StagedChol {
    std::vector<GemmDesc> gram, a, b, d2;
    std::vector<SmallDesc> sd;
    const SmallDesc *dsd = nullptr;
    StagedGemm sg, sa, sb, sc;
    int passes = 0, shifted = 0, kmx = 0;
    size_t nj = 0;
    bool want_r = false;
};

tlr_status stage_cholqr(Ctx &c, std::vector<Job> &jobs, bool on_z, bool want_r, int passes, int shifted,
                        StagedChol &q) {
    const int nb = c.p->nb;
    const size_t nj = jobs.size();
    q.passes = passes;
    q.shifted = shifted;
    q.nj = nj;
    q.want_r = want_r;
    q.kmx = 0;
    for (auto &jb : jobs) q.kmx = std::max(q.kmx, jb.k);
    // every pass forms the Gram matrix of the same panel: one descriptor set;
    // the passes differ only in where R goes
    q.sd.assign((size_t)passes * nj, SmallDesc{});
    for (size_t t = 0; t < nj; ++t) {
        Job &jb = jobs[t];
        double *Yp = on_z ? jb.Zb : jb.Yb;
        q.gram.push_back(gd(Yp, nb, Yp, nb, jb.G, jb.k, jb.k, jb.k, nb, 1.0, 0.0));
        for (int it = 0; it < passes; ++it) {
            SmallDesc d{};
            d.A = jb.G;
            d.lda = jb.k;
            d.R = jb.Rp[it];
            d.ldr = jb.k;
            d.X = jb.T;  // k x k scratch for the Cholesky tiles when they exceed LDS
            d.Y = Yp;
            d.ldy = nb;
            d.m = nb;
            d.k = jb.k;
            d.tile_i = jb.i;
            d.tile_j = jb.j;
            q.sd[(size_t)it * nj + t] = d;
        }
    }
    // the Cholesky factorisation reads only the Gram matrix's lower triangle
    TLR_TRY(stage_gemms(c, true, false, q.gram, &q.sg, true));
    q.dsd = c.push(q.sd);
    if (!q.dsd) return TLR_E_NOMEM;
    if (want_r && passes == 4) {
        // Rt = R4 R3 R2 R1, accumulated through T
        for (auto &jb : jobs) {
            q.a.push_back(gd(jb.Rp[3], jb.k, jb.Rp[2], jb.k, jb.T, jb.k, jb.k, jb.k, jb.k, 1.0, 0.0));
            q.b.push_back(gd(jb.T, jb.k, jb.Rp[1], jb.k, jb.Rt, jb.k, jb.k, jb.k, jb.k, 1.0, 0.0));
            q.d2.push_back(gd(jb.Rt, jb.k, jb.Rp[0], jb.k, jb.T, jb.k, jb.k, jb.k, jb.k, 1.0, 0.0));
        }
        TLR_TRY(stage_gemms(c, false, false, q.a, &q.sa));
        TLR_TRY(stage_gemms(c, false, false, q.b, &q.sb));
        TLR_TRY(stage_gemms(c, false, false, q.d2, &q.sc));
        for (auto &jb : jobs) std::swap(jb.Rt, jb.T);  // the product ends in T
    } else if (want_r && passes == 3) {
        // Rt = R3 R2 R1 through T
        for (auto &jb : jobs) {
            q.a.push_back(gd(jb.Rp[2], jb.k, jb.Rp[1], jb.k, jb.T, jb.k, jb.k, jb.k, jb.k, 1.0, 0.0));
            q.b.push_back(gd(jb.T, jb.k, jb.Rp[0], jb.k, jb.Rt, jb.k, jb.k, jb.k, jb.k, 1.0, 0.0));
        }
        TLR_TRY(stage_gemms(c, false, false, q.a, &q.sa));
        TLR_TRY(stage_gemms(c, false, false, q.b, &q.sb));
    } else if (want_r) {
        return TLR_E_UNSUPPORTED;
    }
    return TLR_OK;
}

tlr_status launch_cholqr(Ctx &c, const StagedChol &q) {
    const int nb = c.p->nb;
    const size_t nj = q.nj;
    for (int it = 0; it < q.passes; ++it) {
        const SmallDesc *dp = q.dsd + (size_t)it * nj;
        const SmallDesc *hp = q.sd.data() + (size_t)it * nj;
        TLR_TRY(launch_staged(c, q.sg));
        TLR_LAUNCH(c, chol_small(dp, (int)nj, q.kmx, it < q.shifted ? 1 : 2, c.params(), c.s, hp));
        TLR_LAUNCH(c, trsm_rows(dp, (int)nj, nb, q.kmx, c.s, hp));
    }
    if (q.want_r) {
        TLR_TRY(launch_staged(c, q.sa));
        TLR_TRY(launch_staged(c, q.sb));
        TLR_TRY(launch_staged(c, q.sc));
    }
    return TLR_OK;
}

// Range finder with one power step:  Y = T W  (W = Gaussian), Q1 = orth(Y);
// Z = T^T Q1, Q2 = orth(Z);  W = T Q2 = Qw Rt, so T ~ Qw Rt Q2^T.  Truncation
// of Rt at tol:
//  * exact_svd: Rt = X S Yr^T (one-sided Jacobi), rank = #{S > tol},
//    U = Qw X_r, V = Q2 (Rt^T X_r)  -- the singular-value rank of the paper;
//  * otherwise: pivoted QR of Rt stopped when the trailing block has
//    Frobenius norm <= tol, Rt ~ Q1 B, U = Qw Q1, V = Q2 B^T (error <= tol,
//    rank at most a few above the singular-value rank, far cheaper).
// Q1 takes two shifted passes while tol >= 1e-12 nb sigma2 (nb sigma2 bounds
// every tile's 2-norm): below about 1e-13 ||T|| two passes leave Q1 too
// ill-conditioned to carry the smallest wanted directions into T^T Q1, and a
// third (deflating) pass restores them.
int q1_passes(const tlr_plan_s *p, double sigma2, double tol) {
    return tol >= 1e-12 * (double)p->nb * sigma2 ? 2 : 3;
}

// Passes for the second and third bases (Q2, and Qw with Rt): one shifted
// and two deflating passes resolve every direction above about 1e-11 of the
// panel's norm, which is enough under the float32 rounding floor of a mixed
// plan (about 1e-7 of the tile's norm); a float64 plan takes two shifted and
// two deflating passes (with three, a smooth field's l at n = 40,000 moved by
// 3e-8 n at tol = 1e-7, above its bound).
int full_passes(const tlr_plan_s *p, double sigma2, double tol) {
    (void)sigma2;
    (void)tol;
    return p->mixed ? 3 : 4;
}

constexpr int kQrSmallSketch = 64;  // widest sketch of the small register QRCP kernel

// `after_first`: called once the first two products of the range finder and
// their bases are queued (the factorisation issues the diagonal tile's
// Cholesky and inverse on the second stream there, ahead of this function's
// own use of that stream, with enough work queued on the main stream to
// cover the host's time for those launches).
tlr_status rsvd(Ctx &c, std::vector<Job> &jobs, double tol, const void *Yj, int Rj, bool exact_svd,
                int passes_q1, int passes_full, const std::function<tlr_status()> *after_first = nullptr) {
    if (jobs.empty()) return TLR_OK;
    // widest sample first: its work-groups, the longest, are dispatched
    // first in every batched launch below (the order of the results is not
    // affected)
    std::stable_sort(jobs.begin(), jobs.end(), [](const Job &a, const Job &b) { return a.k > b.k; });
    const int nb = c.p->nb;
    int kmx = 0;
    for (auto &jb : jobs) kmx = std::max(kmx, jb.k);
    // every descriptor of the wave is staged first and reaches the device in
    // one upload, ahead of the first launch: no copy waits in the stream
    // between two steps of the chain
    StagedApply a1, a2, a3;
    StagedChol q1, q2, q3;
    const int shifted_full = passes_full == 3 ? 1 : 2;
    TLR_TRY(stage_apply(c, jobs, false, true, false, Yj, Rj, a1));              // Yb = T W
    TLR_TRY(stage_cholqr(c, jobs, false, false, passes_q1, 2, q1));             // Yb = Q1 (only its span is used)
    TLR_TRY(stage_apply(c, jobs, true, false, true, Yj, Rj, a2));               // Zb = T^T Q1
    TLR_TRY(stage_cholqr(c, jobs, true, false, passes_full, shifted_full, q2));  // Zb = Q2
    TLR_TRY(stage_apply(c, jobs, false, false, false, Yj, Rj, a3));             // Yb = T Q2
    TLR_TRY(stage_cholqr(c, jobs, false, true, passes_full, shifted_full, q3));  // Yb = Qw, Rt
    // truncation of Rt: sketches of up to 64 columns take the small register
    // kernel, wider ones the larger kernels: when a wave has both, the narrow
    // ones run on the second stream beside the wide ones (a wave is ordered
    // widest first, so the narrow ones form the tail of the list)
    std::vector<SmallDesc> sq;
    std::vector<GemmDesc> gu2, gv2;
    const SmallDesc *dsq = nullptr;
    StagedGemm su, sv;
    size_t nw = 0;
    if (!exact_svd) {
        for (auto &jb : jobs) {
            SmallDesc d{};
            d.A = jb.Rt;
            d.lda = jb.k;
            d.R = jb.G;  // scratch
            d.ldr = jb.k;
            d.X = jb.Xs;
            d.ldx = jb.k;
            d.Y = jb.P;
            d.ldy = jb.k;
            d.rank = jb.stat;
            d.flag = jb.stat + 2;
            d.k = jb.k;
            d.k_full = jb.kfull;
            d.tile_i = jb.i;
            d.tile_j = jb.j;
            d.noise = jb.noise;
            sq.push_back(d);
        }
        while (nw < sq.size() && sq[nw].k > kQrSmallSketch) ++nw;
        dsq = c.push(sq);
        if (!dsq) return TLR_E_NOMEM;
        for (auto &jb : jobs) {
            GemmDesc a = gd(jb.Yb, nb, jb.Xs, jb.k, jb.Uout, nb, nb, 0, jb.k, 1.0, 0.0);
            a.N_dev = jb.stat;
            gu2.push_back(a);
            GemmDesc v = gd(jb.Zb, nb, jb.P, jb.k, jb.Vout, nb, nb, 0, jb.k, 1.0, 0.0);
            v.N_dev = jb.stat;
            gv2.push_back(v);
        }
        TLR_TRY(stage_gemms(c, false, false, gu2, &su, false, c.fc()));
        TLR_TRY(stage_gemms(c, false, false, gv2, &sv, false, c.fc()));
    }
    TLR_TRY(launch_apply(c, a1));
    TLR_TRY(launch_cholqr(c, q1));
    TLR_TRY(launch_apply(c, a2));
    TLR_TRY(launch_cholqr(c, q2));
    if (after_first) TLR_TRY((*after_first)());
    TLR_TRY(launch_apply(c, a3));
    TLR_TRY(launch_cholqr(c, q3));
    if (!exact_svd) {
        if (nw > 0 && nw < sq.size()) {
            TLR_TRY(c.flush());
            hipStream_t ss = c.fork();
            TLR_TRY(qrcp_trunc(dsq + nw, (int)(sq.size() - nw), kQrSmallSketch, tol, c.p->min_tail, c.p->kmax,
                               c.p->rcap, c.params(), ss));
            TLR_TRY(qrcp_trunc(dsq, (int)nw, kmx, tol, c.p->min_tail, c.p->kmax, c.p->rcap, c.params(), c.s,
                               kQrSmallSketch + 1));
            TLR_TRY(c.join());
        } else {
            TLR_LAUNCH(c, qrcp_trunc(dsq, (int)sq.size(), kmx, tol, c.p->min_tail, c.p->kmax, c.p->rcap, c.params(),
                                     c.s));
        }
        TLR_TRY(launch_staged(c, su));
        return launch_staged(c, sv);
    }
    std::vector<SmallDesc> sd;
    for (auto &jb : jobs) {
        SmallDesc d{};
        d.A = jb.Rt;
        d.lda = jb.k;
        d.R = jb.G;  // scratch
        d.ldr = jb.k;
        d.X = jb.Xs;
        d.ldx = jb.k;
        d.S = jb.S;
        d.rank = jb.stat;
        d.flag = jb.stat + 2;
        d.k = jb.k;
        d.k_full = jb.kfull;
        d.tile_i = jb.i;
        d.tile_j = jb.j;
        sd.push_back(d);
    }
    TLR_PUSH(dsd, c, sd);
    TLR_LAUNCH(c, jacobi_svd(dsd, (int)sd.size(), kmx, tol, c.p->min_tail, c.p->kmax, c.p->rcap, c.params(), c.s));
    std::vector<GemmDesc> gu, gp, gv;
    for (auto &jb : jobs) {
        GemmDesc a = gd(jb.Yb, nb, jb.Xs, jb.k, jb.Uout, nb, nb, 0, jb.k, 1.0, 0.0);
        a.N_dev = jb.stat;
        gu.push_back(a);
        GemmDesc b = gd(jb.Rt, jb.k, jb.Xs, jb.k, jb.P, jb.k, jb.k, 0, jb.k, 1.0, 0.0);
        b.N_dev = jb.stat;
        gp.push_back(b);
        GemmDesc v = gd(jb.Zb, nb, jb.P, jb.k, jb.Vout, nb, nb, 0, jb.k, 1.0, 0.0);
        v.N_dev = jb.stat;
        gv.push_back(v);
    }
    TLR_TRY(launch_gemms(c, false, false, gu, c.fc()));
    TLR_TRY(launch_gemms(c, true, false, gp));
    TLR_TRY(launch_gemms(c, false, false, gv, c.fc()));
    return TLR_OK;
}

// Tiles kept dense: U <- D (nb x nb), V <- I, host flag set.  Stream-ordered
// after whatever produced D.
tlr_status make_dense(Ctx &c, const std::vector<std::pair<int, int>> &tiles, const std::vector<const double *> &src) {
    if (tiles.empty()) return TLR_OK;
    const int nb = c.p->nb;
    std::vector<CopyDesc> cps;
    std::vector<double *> ids;
    for (size_t q = 0; q < tiles.size(); ++q) {
        const int i = tiles[q].first, j = tiles[q].second;
        cps.push_back(CopyDesc{src[q], c.wideU(i, j), (int64_t)nb * nb, 0});
        ids.push_back(c.wideV(i, j));
        c.dflag[(size_t)i * c.p->nt + j] = 1;
    }
    TLR_PUSH(dcp, c, cps);
    TLR_LAUNCH(c, copy_batched(dcp, (int)cps.size(), (int64_t)nb * nb, c.s));
    TLR_PUSH(did, c, ids);
    TLR_LAUNCH(c, identity_batched(did, (int)ids.size(), nb, c.s));
    return TLR_OK;
}

int tile_rows(const tlr_plan_s *p, int i) {
    const int64_t r = p->n - (int64_t)i * p->nb;
    return (int)std::min<int64_t>(r, p->nb);
}

int clamp_k(const tlr_plan_s *p, int want, int kfull) {
    int cap = std::min(p->kmax, kfull);
    int k = std::max(want, std::min(p->k0, cap));
    k = (k + 7) / 8 * 8;
    return std::max(1, std::min(k, cap));
}

// Smallest ladder width >= want (see widen_k).
int ladder_k(const tlr_plan_s *p, int want, int kfull) {
    static const int ladder[] = {32, 64, 112, 176, 192, 240, 320, 400, 512};
    int k = want;
    for (int w : ladder)
        if (w >= want) {
            k = w;
            break;
        }
    return clamp_k(p, k, kfull);
}

// Next sketch width after a too-narrow sample: a fixed ladder that stays at
// the widths the small kernels handle in LDS as long as possible.
int widen_k(const tlr_plan_s *p, int k, int kfull) {
    static const int ladder[] = {32, 64, 112, 176, 192, 240, 320, 400, 512};
    int next = 2 * k;
    for (int w : ladder)
        if (w > k) {
            next = w;
            break;
        }
    return std::max(clamp_k(p, next, kfull), std::min(k, std::min(p->kmax, kfull)));
}

}  // namespace

void note_pinned_alloc() { g_pinned_allocs.fetch_add(1, std::memory_order_relaxed); }
void note_stream_created() { g_streams_created.fetch_add(1, std::memory_order_relaxed); }
void alloc_counts(int64_t *pinned, int64_t *streams) {
    *pinned = g_pinned_allocs.load(std::memory_order_relaxed);
    *streams = g_streams_created.load(std::memory_order_relaxed);
}

// ------------------------------------------------------------------ plan --

tlr_status plan_create(tlr_plan *out, int64_t n, int nb, int maxrank, tlr_precision prec, uint32_t flags) {
    if (!out) return TLR_E_INVAL;
    *out = nullptr;
    if (n < 1 || nb < 16 || nb > 4096) return TLR_E_INVAL;
    if (prec != TLR_FP64 && prec != TLR_MIXED_FP32) return TLR_E_INVAL;
    // float32 factors: the pivoted-QR truncation with its rounding floor only
    // (no dense off-diagonal tiles, no singular-value truncation)
    if (prec == TLR_MIXED_FP32 && (flags & (TLR_PLAN_DENSE_TILES | TLR_PLAN_SVD_TRUNCATION)))
        return TLR_E_UNSUPPORTED;
    auto *p = new tlr_plan_s{};
    p->n = n;
    p->nb = nb;
    p->nt = (int)cdiv(n, nb);
    p->npad = (int64_t)p->nt * nb;
    p->ntiles = (int64_t)p->nt * (p->nt - 1) / 2;
    p->pover = 8;  // sketch width for a recompression: previous rank + 8 (the tail test's margin)
    p->min_tail = 8;
    p->k0 = 32;
    int rcap = (maxrank <= 0) ? nb / 2 : std::min(maxrank, nb);
    rcap = std::max(1, std::min(rcap, kMaxSketch - p->pover));
    p->rcap = rcap;
    p->kmax = std::min({nb, rcap + p->pover, kMaxSketch});
    p->prec = prec;
    p->flags = flags;
    p->mixed = prec == TLR_MIXED_FP32;
    p->fw = p->mixed ? (int)sizeof(float) : (int)sizeof(double);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(std::max<size_t>(bytes, 1), 256);
        return o;
    };
    p->off_params = take(sizeof(ParamsBlock));
    p->off_x = take(sizeof(double) * p->npad);
    p->off_y = take(sizeof(double) * p->npad);
    p->off_diag = take(sizeof(double) * (size_t)p->nt * nb * nb);
    p->off_rsig = take(sizeof(int32_t) * (size_t)p->nt * p->nt);
    p->off_rL = take(sizeof(int32_t) * (size_t)p->nt * p->nt);
    p->off_tstat = take(sizeof(int32_t) * 4 * (size_t)std::max<int64_t>(p->ntiles, 1));
    p->off_tofs = take(sizeof(int64_t) * 2 * ((size_t)std::max<int64_t>(p->ntiles, 1) + 1));
    p->off_nrm_s = take(sizeof(double) * (size_t)p->nt * p->nt);
    p->off_nrm_l = take(sizeof(double) * (size_t)p->nt * p->nt);
    p->off_noise = take(sizeof(double) * (size_t)std::max<int64_t>(p->ntiles, 1));
    p->off_linv = take(sizeof(double) * (size_t)p->nt * nb * nb);  // L_jj^-1 of every tile column
    p->dense_ok = (flags & TLR_PLAN_DENSE_TILES) != 0;
    p->svd_trunc = (flags & TLR_PLAN_SVD_TRUNCATION) != 0;
    p->off_dense = take(sizeof(int32_t) * (size_t)p->nt * p->nt);
    p->off_wide = p->dense_ok ? take(sizeof(double) * 2 * (size_t)nb * nb * (size_t)std::max<int64_t>(p->ntiles, 1)) : 0;
    p->off_yvec = take(sizeof(double) * p->npad);
    p->off_ysol = take(sizeof(double) * p->npad);
    p->off_omega = take(sizeof(double) * (size_t)nb * p->kmax);
    p->off_knu = take(sizeof(double) * 3 * kChebPieces * (kChebDeg + 1));  // three for the bivariate model
    // descriptors of one wave: about 42 (GEMM and small-kernel descriptors,
    // ~100 bytes each) per job of a full kMaxWave-job wave, plus the
    // per-column products of the factorisation
    p->desc_bytes = 32u << 20;
    p->off_desc = take(p->desc_bytes);
    // arena: one full wave of dense-tile jobs, plus the factorisation's
    // per-column panels, bounded to keep small problems small
    const size_t per_job = job_words(nb, p->kmax, rcap, 0, true) * sizeof(double);
    const size_t col_panels =
        sizeof(double) * (size_t)nb * (size_t)std::max(1, p->nt - 1) * ((flags & TLR_PLAN_DENSE_TILES) ? nb : rcap) * 3;
    // a factorisation job at the rank cap everywhere: X_i (nb x R), the
    // Schur buffers (R = (nt-1) maxrank) and its M_ik blocks
    const int64_t rmax = (int64_t)std::max(1, p->nt - 1) * (p->dense_ok ? nb : rcap);
    const size_t potrf_job =
        (job_words(nb, p->kmax, rcap, (int)std::min<int64_t>(rmax, 1 << 30), false) + (size_t)nb * rmax +
         (size_t)std::max(1, p->nt - 1) * (p->dense_ok ? (size_t)nb * nb : (size_t)rcap * rcap) +
         (p->dense_ok ? 3 * (size_t)nb * nb : 0)) * sizeof(double);
    size_t arena = std::max<size_t>(per_job * (size_t)std::min<int64_t>(std::max<int64_t>(p->ntiles, 1), 64),
                                    col_panels + potrf_job * 2);
    arena = std::max<size_t>(arena, 64u << 20);
    arena = std::min<size_t>(arena, (size_t)16 << 30);
    p->arena_bytes = arena;
    p->off_arena = take(arena);
    // the factor arena runs to the end of the caller's workspace; the default
    // size holds a slot of maxrank columns for every tile
    p->off_fac = off;
    p->ws_bytes = off + align_up((size_t)p->fw * 2 * (size_t)nb * rcap * (size_t)p->ntiles, 256);
    *out = p;
    return TLR_OK;
}

void plan_destroy(tlr_plan p) { delete p; }

size_t plan_ws_bytes(tlr_plan p) { return p ? p->ws_bytes : 0; }

size_t plan_ws_bytes_budget(tlr_plan p, int64_t rank_budget) {
    if (!p) return 0;
    if (rank_budget <= 0) return p->ws_bytes;
    return p->off_fac + align_up((size_t)p->fw * 2 * (size_t)p->nb * (size_t)rank_budget, 256);
}

// ------------------------------------------------------------ generation --

tlr_status gen_tiles(tlr_plan p, const double *d_locs, tlr_theta th, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!p || !d_locs || !d_ws) return TLR_E_INVAL;
    if (ws_bytes < p->off_fac) return TLR_E_NOMEM;
    MaternConst mc{};
    if (!make_matern_const(th.sigma2, th.beta, th.nu, &mc)) return TLR_E_INVAL;
    Ctx c(p, d_ws, s);
    TLR_TRY(build_knu_table(&mc, reinterpret_cast<double *>(c.ws + p->off_knu), s));
    ParamsBlock hb{};
    TLR_HIP(hipMemcpyAsync(&hb, c.pblock(), sizeof(ParamsBlock), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    const uint64_t keep_magic = hb.hint_magic;
    hb = ParamsBlock{};
    hb.dp.sigma2 = th.sigma2;
    hb.dp.beta = th.beta;
    hb.dp.nu = th.nu;
    hb.dp.status = 0;
    hb.dp.fail_i = hb.dp.fail_j = -1;
    hb.dp.dense_ok = p->dense_ok ? 1 : 0;
    // float32 factors carry rounding noise of about 2^-24 of their norm: the
    // truncation floor is twice that (the sum of the two factors' roundings)
    hb.dp.floor_rel = p->mixed ? 2.0 * 0x1.0p-24 : 0.0;
    hb.mc = mc;
    hb.hint_magic = keep_magic;
    TLR_HIP(hipMemcpyAsync(c.pblock(), &hb, sizeof(ParamsBlock), hipMemcpyHostToDevice, s));
    TLR_TRY(split_locs(d_locs, p->n, p->npad, c.x(), c.y(), s));
    std::vector<GenDesc> g;
    for (int k = 0; k < p->nt; ++k) g.push_back(GenDesc{c.diag(k), k * p->nb, k * p->nb, p->nb, 1});
    TLR_PUSH(dg, c, g);
    TLR_LAUNCH(c, gen_tiles_launch(dg, (int)g.size(), p->nb, p->n, c.x(), c.y(), mc, s));
    TLR_TRY(gaussian_fill(c.omega(), (int64_t)p->nb * p->kmax, kSketchSeed, s));
    TLR_HIP(hipStreamSynchronize(s));  // host descriptors above go out of scope
    return TLR_OK;
}

// The parsimonious bivariate Matern model: the plan's n is the matrix size,
// twice the number of locations; entry 2p + v is variable v at location p.
tlr_status gen_tiles_bivariate(tlr_plan p, const double *d_locs, const tlr_theta_biv &th, void *d_ws, size_t ws_bytes,
                               hipStream_t s) {
    if (!p || !d_locs || !d_ws || p->n % 2 != 0) return TLR_E_INVAL;
    if (ws_bytes < p->off_fac) return TLR_E_NOMEM;
    BivConst bc{};
    if (!make_biv_const(th.sigma2_11, th.sigma2_22, th.a, th.nu_11, th.nu_22, th.beta_12, &bc)) return TLR_E_INVAL;
    Ctx c(p, d_ws, s);
    double *tabs = reinterpret_cast<double *>(c.ws + p->off_knu);
    for (int q = 0; q < 3; ++q) TLR_TRY(build_knu_table(&bc.m[q], tabs + (size_t)q * kChebPieces * (kChebDeg + 1), s));
    ParamsBlock hb{};
    TLR_HIP(hipMemcpyAsync(&hb, c.pblock(), sizeof(ParamsBlock), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    const uint64_t keep_magic = hb.hint_magic;
    hb = ParamsBlock{};
    // the larger variance bounds every tile's norm (nb sigma2), as in the
    // univariate model: the range finder's pass rule reads it
    hb.dp.sigma2 = std::max(th.sigma2_11, th.sigma2_22);
    hb.dp.beta = th.a;
    hb.dp.nu = std::min(th.nu_11, th.nu_22);
    hb.dp.status = 0;
    hb.dp.fail_i = hb.dp.fail_j = -1;
    hb.dp.dense_ok = p->dense_ok ? 1 : 0;
    hb.dp.floor_rel = p->mixed ? 2.0 * 0x1.0p-24 : 0.0;
    hb.mc = bc.m[0];
    hb.bv = bc;
    hb.hint_magic = keep_magic;
    TLR_HIP(hipMemcpyAsync(c.pblock(), &hb, sizeof(ParamsBlock), hipMemcpyHostToDevice, s));
    TLR_TRY(split_locs(d_locs, p->n / 2, p->npad, c.x(), c.y(), s));
    std::vector<GenDesc> g;
    for (int k = 0; k < p->nt; ++k) g.push_back(GenDesc{c.diag(k), k * p->nb, k * p->nb, p->nb, 1});
    TLR_PUSH(dg, c, g);
    TLR_LAUNCH(c, gen_tiles_biv_launch(dg, (int)g.size(), p->nb, p->n, c.x(), c.y(), bc, s));
    TLR_TRY(gaussian_fill(c.omega(), (int64_t)p->nb * p->kmax, kSketchSeed, s));
    TLR_HIP(hipStreamSynchronize(s));  // host descriptors above go out of scope
    return TLR_OK;
}

// ------------------------------------------------------------ compression --

tlr_status compress(tlr_plan p, double tol, void *d_ws, size_t ws_bytes, int32_t *d_ranks, hipStream_t s) {
    if (!p || !d_ws) return TLR_E_INVAL;
    if (!(tol >= 0.0) || !std::isfinite(tol)) return TLR_E_INVAL;
    if (ws_bytes < p->off_fac) return TLR_E_NOMEM;
    Ctx c(p, d_ws, s);
    c.ws_size = ws_bytes;
    c.reset_slots();
    const int nt = p->nt, nb = p->nb;
    ParamsBlock hb{};
    TLR_HIP(hipMemcpyAsync(&hb, c.pblock(), sizeof(ParamsBlock), hipMemcpyDeviceToHost, s));
    std::vector<int32_t> hint((size_t)nt * nt, -1), ranks((size_t)nt * nt, 0);
    TLR_HIP(hipMemcpyAsync(hint.data(), c.rsig(), sizeof(int32_t) * hint.size(), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    c.dflag.assign((size_t)nt * nt, 0);  // every tile starts low-rank
    // Every tile starts from the same sketch width (no state carried between
    // evaluations), so the result depends on the inputs only.
    const bool hints_ok = false;
    const MaternConst mc = hb.mc;
    const BivConst bv = hb.bv;
    {
        double t = tol;
        TLR_HIP(hipMemcpyAsync(&c.pblock()->tol, &t, sizeof(double), hipMemcpyHostToDevice, s));
        TLR_HIP(hipStreamSynchronize(s));
    }
    struct Pending {
        int i, j, k;
    };
    std::vector<Pending> pending;
    bool arena_full = false;  // a factor did not fit the arena: stop (status set)
    for (int i = 1; i < nt; ++i)
        for (int j = 0; j < i; ++j) {
            const int kfull = std::min(tile_rows(p, i), tile_rows(p, j));
            const int h = hints_ok ? hint[(size_t)i * nt + j] : -1;
            const int want = (h >= 0) ? h + p->pover : p->k0;
            pending.push_back({i, j, clamp_k(p, want, kfull)});
        }
    while (!pending.empty() && !arena_full) {
        std::vector<Pending> retry;
        size_t pos = 0;
        while (pos < pending.size() && !arena_full) {
            c.arena_used = 0;
            c.use_free_tail();
            std::vector<Job> jobs;
            std::vector<GenDesc> gens;
            while (pos < pending.size()) {
                const Pending &pt = pending[pos];
                const size_t need = job_words(nb, pt.k, 0, 0, true) * sizeof(double);
                if (c.arena_used + need > c.arena_cap && !jobs.empty()) break;
                Job jb{};
                jb.i = pt.i;
                jb.j = pt.j;
                jb.k = pt.k;
                jb.kfull = std::min(tile_rows(p, pt.i), tile_rows(p, pt.j));
                double *A = c.alloc((size_t)nb * nb);
                if (!A || !alloc_job(c, jb, 0)) return TLR_E_NOMEM;
                jb.A = A;
                // results go to their slot once the rank is known
                jb.Uout = c.alloc_fac((size_t)nb * pt.k);
                jb.Vout = c.alloc_fac((size_t)nb * pt.k);
                if (!jb.Uout || !jb.Vout) return TLR_E_NOMEM;
                jb.stat = c.tstat(tile_index(pt.i, pt.j));
                gens.push_back(GenDesc{A, pt.i * nb, pt.j * nb, nb, 0});
                jobs.push_back(jb);
                ++pos;
                if (jobs.size() >= (size_t)kMaxWave) break;
            }
            TLR_PUSH(dg, c, gens);
            if (bv.on)
                TLR_LAUNCH(c, gen_tiles_biv_launch(dg, (int)gens.size(), nb, p->n, c.x(), c.y(), bv, s));
            else
                TLR_LAUNCH(c, gen_tiles_launch(dg, (int)gens.size(), nb, p->n, c.x(), c.y(), mc, s));
            TLR_TRY(rsvd(c, jobs, tol, nullptr, 0, p->svd_trunc, q1_passes(p, hb.dp.sigma2, tol),
                         full_passes(p, hb.dp.sigma2, tol)));
            Ctx::StatRead sr;
            TLR_TRY(c.read_stats(jobs, sr));
            TLR_TRY(c.sync_reset());
            std::vector<int32_t> st(4 * jobs.size());
            for (size_t q = 0; q < jobs.size(); ++q)
                std::memcpy(&st[4 * q], &sr.raw[(size_t)(tile_index(jobs[q].i, jobs[q].j) - sr.t0) * 4],
                            4 * sizeof(int32_t));
            if (debug_enabled()) {
                int code = 0;
                TLR_TRY(c.read_status(&code));
                for (size_t q = 0; q < jobs.size(); ++q)
                    std::fprintf(stderr, "compress tile (%d,%d) k=%d write=%d num=%d flag=%d status=%d\n", jobs[q].i,
                                 jobs[q].j, jobs[q].k, st[4 * q], st[4 * q + 1], st[4 * q + 2], code);
            }
            std::vector<std::pair<int, int>> dz;
            std::vector<const double *> dsrc;
            std::vector<CopyDesc> put;
            int64_t put_max = 0;
            for (size_t q = 0; q < jobs.size(); ++q) {
                const Job &jb = jobs[q];
                if (st[4 * q + 2]) {
                    retry.push_back({jb.i, jb.j, widen_k(p, jb.k, jb.kfull)});
                } else {
                    const int num = st[4 * q + 1];
                    int rk = st[4 * q];
                    if (num > p->rcap) {
                        rk = -1;
                        if (p->dense_ok) {  // keep the generated tile dense
                            dz.emplace_back(jb.i, jb.j);
                            dsrc.push_back(jb.A);
                            rk = nb;
                        }
                    } else if (rk > 0) {
                        if (!c.take_slot(jb.i, jb.j, rk)) {
                            if (!arena_full) TLR_TRY(c.host_fail(TLR_ARENA_OVERFLOW, jb.i, jb.j));
                            arena_full = true;
                        } else {
                            put.push_back(CopyDesc{jb.Uout, c.U(jb.i, jb.j), (int64_t)nb * rk, p->mixed ? 2 : 0});
                            put.push_back(CopyDesc{jb.Vout, c.V(jb.i, jb.j), (int64_t)nb * rk, p->mixed ? 2 : 0});
                            put_max = std::max<int64_t>(put_max, (int64_t)nb * rk);
                        }
                    }
                    ranks[(size_t)jb.i * nt + jb.j] = rk;
                }
            }
            // into their slots before the next wave reuses the job buffers
            if (!put.empty()) {
                TLR_PUSH(dput, c, put);
                TLR_LAUNCH(c, copy_batched(dput, (int)put.size(), put_max, s));
            }
            // before the next wave reuses the arena that holds the tiles
            TLR_TRY(make_dense(c, dz, dsrc));
        }
        pending.swap(retry);
    }
    if (p->mixed && p->ntiles > 0 && !arena_full) {
        // ||V_ij||_F = ||U_ij V_ij^T||_F (U has orthonormal columns): the
        // scale of each stored tile's float32 rounding
        std::vector<NormDesc> nd;
        for (int i = 1; i < nt; ++i)
            for (int j = 0; j < i; ++j)
                nd.push_back(NormDesc{static_cast<const float *>(c.V(i, j)), c.tstat(tile_index(i, j)),
                                      c.nrm_s() + (size_t)i * nt + j});
        TLR_PUSH(dnd, c, nd);
        TLR_LAUNCH(c, factor_norms(dnd, (int)nd.size(), nb, s));
    }
    TLR_TRY(c.store_dense());
    TLR_TRY(c.store_slots());
    TLR_HIP(hipMemcpyAsync(c.rsig(), ranks.data(), sizeof(int32_t) * ranks.size(), hipMemcpyHostToDevice, s));
    TLR_HIP(hipMemcpyAsync(c.rL(), ranks.data(), sizeof(int32_t) * ranks.size(), hipMemcpyHostToDevice, s));
    std::vector<int32_t> out_ranks = ranks;
    for (size_t t = 0; t < out_ranks.size(); ++t)
        if (c.dflag[t]) out_ranks[t] = -2;
    if (d_ranks)
        TLR_HIP(hipMemcpyAsync(d_ranks, out_ranks.data(), sizeof(int32_t) * out_ranks.size(), hipMemcpyHostToDevice,
                               s));
    const uint64_t magic = kHintMagic;
    TLR_HIP(hipMemcpyAsync(&c.pblock()->hint_magic, &magic, sizeof(magic), hipMemcpyHostToDevice, s));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
}

// ------------------------------------------------------- factorisation --

tlr_status potrf(tlr_plan p, void *d_ws, size_t ws_bytes, hipStream_t s) {
    if (!p || !d_ws) return TLR_E_INVAL;
    if (ws_bytes < p->off_fac) return TLR_E_NOMEM;
    Ctx c(p, d_ws, s);
    const int nt = p->nt, nb = p->nb;
    ParamsBlock hb{};
    std::vector<int32_t> r((size_t)nt * nt, 0);
    TLR_HIP(hipMemcpyAsync(&hb, c.pblock(), sizeof(ParamsBlock), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipMemcpyAsync(r.data(), c.rL(), sizeof(int32_t) * r.size(), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    const double tol = hb.tol;
    if (hb.dp.status != 0) return TLR_OK;  // already failed: l = -inf
    c.ws_size = ws_bytes;
    TLR_TRY(c.load_dense());
    TLR_TRY(c.load_slots());
    for (int i = 0; i < nt; ++i)
        for (int j = 0; j < i; ++j)
            if (r[(size_t)i * nt + j] < 0) return TLR_OK;  // overflow recorded by compress
    // a failure recorded on the device (a pivot lost, an arena overflow) is
    // seen at the next status read-back; the factorisation then stops
    bool failed = false;
    for (int j = 0; j < nt; ++j) {
        c.arena_used = 0;
        int Rj = 0;
        std::vector<int> off(j + 1, 0);
        for (int k = 0; k < j; ++k) {
            off[k] = Rj;
            Rj += r[(size_t)j * nt + k];
        }
        void *Yj = nullptr;
        if (Rj > 0) {
            // Yj = [U_j0 | ... | U_j,j-1]; Xd = [U_jk (V_jk^T V_jk)]_k; D_j -= Xd Yj^T
            // (both panels in the factors' element type)
            Yj = c.alloc_fac((size_t)nb * Rj);
            void *Xd = c.alloc_fac((size_t)nb * Rj);
            size_t msz = 0;
            for (int k = 0; k < j; ++k) msz += (size_t)r[(size_t)j * nt + k] * r[(size_t)j * nt + k];
            double *Md = c.alloc(std::max<size_t>(msz, 1));
            if (!Yj || !Xd || !Md) return TLR_E_NOMEM;
            std::vector<GemmDesc> gm, gx;
            std::vector<SmallDesc> cp;
            size_t mo = 0;
            for (int k = 0; k < j; ++k) {
                const int rk = r[(size_t)j * nt + k];
                if (rk == 0) continue;
                gm.push_back(gd(c.V(j, k), nb, c.V(j, k), nb, Md + mo, rk, rk, rk, nb, 1.0, 0.0));
                gx.push_back(gd(c.U(j, k), nb, Md + mo, rk, c.fac_at(Xd, (size_t)off[k] * nb), nb, nb, rk, rk, 1.0, 0.0));
                mo += (size_t)rk * rk;
            }
            TLR_TRY(launch_gemms(c, true, false, gm, c.fa() | c.fb()));
            TLR_TRY(launch_gemms(c, false, false, gx, c.fa() | c.fc()));
            // gather Yj: U_jk occupies the first r_jk columns of its slot (ld nb)
            std::vector<CopyDesc> cps;
            int64_t mxw = 0;
            for (int k = 0; k < j; ++k) {
                const int rk = r[(size_t)j * nt + k];
                if (rk == 0) continue;
                cps.push_back(CopyDesc{c.U(j, k), c.fac_at(Yj, (size_t)off[k] * nb), (int64_t)rk * nb, p->mixed ? 2 : 0});
                mxw = std::max<int64_t>(mxw, (int64_t)rk * nb);
            }
            TLR_PUSH(dcp, c, cps);
            TLR_LAUNCH(c, copy_batched(dcp, (int)cps.size(), mxw, s));
            std::vector<GemmDesc> gdg{gd(Xd, nb, Yj, nb, c.diag(j), nb, nb, nb, Rj, -1.0, 1.0)};
            TLR_TRY(launch_gemms(c, false, true, gdg, c.fa() | c.fb()));
        }
        // dense Cholesky of the updated diagonal tile, beside the
        // recompression of the tiles below (which never reads it); only the
        // triangular solves at the end of the column need its factor.  The
        // side stream is forked here, after the diagonal update; its launches
        // are issued once the main stream has the column's first batch of
        // work queued, so that their host-side cost does not starve it.
        // After the factor, the same stream forms its inverse (L_jj X = I by
        // the blocked substitution), which turns the triangular solves at the
        // end of the column into one product; the forward solve of the
        // likelihood uses it again.
        hipStream_t side_s = nullptr;
        const GemmDesc *dpd = nullptr;
        SmallDesc inv_sd{};
        const SmallDesc *dinv_sd = nullptr;
        GemmDesc *dinv_g = nullptr;
        double *const *dinv_id = nullptr;
        {
            std::vector<GemmDesc> pd((size_t)cdiv(nb, 64));
            potrf_tile_descs(c.diag(j), nb, pd.data());
            dpd = c.push(pd);
            if (!dpd) return TLR_E_NOMEM;
            inv_sd.Y = c.linv(j);
            inv_sd.ldy = nb;
            inv_sd.k = nb;
            std::vector<GemmDesc> ig((size_t)cdiv(nb, 64));
            trsm_left_lower_descs(c.diag(j), nb, &inv_sd, 1, ig.data(), false);
            dinv_g = c.push(ig);
            dinv_sd = c.push(&inv_sd, 1);
            double *const idp[1] = {c.linv(j)};
            dinv_id = c.push(idp, 1);
            if (!dinv_g || !dinv_sd || !dinv_id) return TLR_E_NOMEM;
            TLR_TRY(c.flush());
            side_s = c.fork();
        }
        bool diag_issued = false;
        const std::function<tlr_status()> issue_diag = [&]() -> tlr_status {
            if (diag_issued) return TLR_OK;
            diag_issued = true;
            TLR_TRY(potrf_tile(c.diag(j), nb, j, c.params(), dpd, side_s));
            TLR_TRY(identity_batched(dinv_id, 1, nb, side_s));
            return trsm_left_lower(c.diag(j), nb, dinv_sd, &inv_sd, 1, nb, dinv_g, nullptr, side_s, false);
        };
        // Schur complement of the tiles below, re-compressed once
        std::vector<int> rows;
        for (int i = j + 1; i < nt; ++i) rows.push_back(i);
        if (Rj > 0 && !rows.empty()) {
            const size_t mark = c.arena_used;
            std::vector<int> todo = rows;
            std::vector<int> kk(nt, 0);
            for (int i : todo) {
                const int kfull = std::min(tile_rows(p, i), tile_rows(p, j));
                kk[i] = ladder_k(p, r[(size_t)i * nt + j] + p->pover, kfull);
            }
            while (!todo.empty() && !failed) {
                std::vector<int> retry;
                size_t pos = 0;
                while (pos < todo.size()) {
                    c.arena_used = mark;
                    std::vector<Job> jobs;   // low-rank tiles: recompressed by the range finder
                    std::vector<Job> djobs;  // dense tiles: Schur complement formed explicitly
                    std::vector<GemmDesc> gmm, gxx;
                    while (pos < todo.size()) {
                        const int i = todo[pos];
                        const int rij = r[(size_t)i * nt + j];
                        const bool dz = c.dense(i, j);
                        size_t msz = 0;
                        for (int k = 0; k < j; ++k) msz += (size_t)r[(size_t)i * nt + k] * r[(size_t)j * nt + k];
                        size_t words = (size_t)nb * Rj + msz + 64;
                        if (dz)
                            words += (size_t)nb * nb + 64;
                        else
                            words += job_words(nb, kk[i], rij, Rj, false) + (p->dense_ok ? (size_t)nb * nb + 256 : 0);
                        if (c.arena_used + words * sizeof(double) > c.arena_cap && !(jobs.empty() && djobs.empty()))
                            break;
                        Job jb{};
                        jb.i = i;
                        jb.j = j;
                        jb.k = kk[i];
                        jb.kfull = std::min(tile_rows(p, i), tile_rows(p, j));
                        jb.r = rij;
                        jb.Uop = c.U(i, j);
                        jb.Vop = c.V(i, j);
                        void *Xi = c.alloc_fac((size_t)nb * Rj);
                        if (!Xi) return TLR_E_NOMEM;
                        jb.Xi = Xi;
                        jb.stat = c.tstat(tile_index(i, j));
                        if (dz) {
                            jb.D = c.alloc((size_t)nb * nb);
                            if (!jb.D) return TLR_E_NOMEM;
                        } else {
                            if (!alloc_job(c, jb, Rj)) return TLR_E_NOMEM;
                            // results land in temporaries and go to the tile's slot once
                            // the rank is known; the old factors stay intact meanwhile
                            // (a retry, or the dense form, still reads them)
                            jb.Uout = c.alloc_fac((size_t)nb * jb.k);
                            jb.Vout = c.alloc_fac((size_t)nb * jb.k);
                            if (!jb.Uout || !jb.Vout) return TLR_E_NOMEM;
                            if (p->dense_ok) {
                                jb.D = c.alloc((size_t)nb * nb);
                                if (!jb.D) return TLR_E_NOMEM;
                            }
                        }
                        // X_i blocks: U_ik (V_ik^T V_jk)
                        double *Mik = c.alloc(std::max<size_t>(msz, 1));
                        if (!Mik) return TLR_E_NOMEM;
                        size_t mo = 0;
                        for (int k = 0; k < j; ++k) {
                            const int rik = r[(size_t)i * nt + k], rjk = r[(size_t)j * nt + k];
                            if (rjk == 0) continue;
                            if (rik == 0) {
                                // zero block of X_i
                                gxx.push_back(gd(c.U(i, k), nb, Mik, 1, c.fac_at(Xi, (size_t)off[k] * nb), nb, nb, rjk, 0,
                                                 1.0, 0.0));
                                continue;
                            }
                            gmm.push_back(gd(c.V(i, k), nb, c.V(j, k), nb, Mik + mo, rik, rik, rjk, nb, 1.0, 0.0));
                            gxx.push_back(gd(c.U(i, k), nb, Mik + mo, rik, c.fac_at(Xi, (size_t)off[k] * nb), nb, nb, rjk, rik,
                                             1.0, 0.0));
                            mo += (size_t)rik * rjk;
                        }
                        (dz ? djobs : jobs).push_back(jb);
                        ++pos;
                        if (jobs.size() + djobs.size() >= (size_t)kMaxWave) break;
                    }
                    TLR_TRY(launch_gemms(c, true, false, gmm, c.fa() | c.fb()));
                    TLR_TRY(launch_gemms(c, false, false, gxx, c.fa() | c.fc()));
                    // explicit Schur complement D = U V^T - X_i Y_j^T of a tile (dense or converting)
                    auto schur_dense = [&](const std::vector<Job> &js) -> tlr_status {
                        std::vector<GemmDesc> g1, g2;
                        for (const Job &jb : js) {
                            g1.push_back(gd(jb.Uop, nb, jb.Vop, nb, jb.D, nb, nb, nb, jb.r, 1.0, 0.0));
                            g2.push_back(gd(jb.Xi, nb, Yj, nb, jb.D, nb, nb, nb, Rj, -1.0, 1.0));
                        }
                        TLR_TRY(launch_gemms(c, false, true, g1, c.fa() | c.fb()));
                        return launch_gemms(c, false, true, g2, c.fa() | c.fb());
                    };
                    if (!djobs.empty()) {
                        TLR_TRY(schur_dense(djobs));
                        std::vector<std::pair<int, int>> dt;
                        std::vector<const double *> ds;
                        for (const Job &jb : djobs) {
                            dt.emplace_back(jb.i, jb.j);
                            ds.push_back(jb.D);
                        }
                        TLR_TRY(make_dense(c, dt, ds));
                    }
                    if (!jobs.empty() && p->mixed) {
                        // float32 rounding noise of each Schur operator, for the truncation floor
                        std::vector<NoiseDesc> nz;
                        for (Job &jb : jobs) {
                            jb.noise = c.noise(tile_index(jb.i, jb.j));
                            nz.push_back(NoiseDesc{jb.i, jb.j, c.noise(tile_index(jb.i, jb.j))});
                        }
                        TLR_PUSH(dnz, c, nz);
                        TLR_LAUNCH(c, schur_noise(dnz, (int)nz.size(), nt, c.nrm_s(), c.nrm_l(), s));
                    }
                    if (!jobs.empty())
                        TLR_TRY(rsvd(c, jobs, tol, Yj, Rj, p->svd_trunc, q1_passes(p, hb.dp.sigma2, tol),
                                     full_passes(p, hb.dp.sigma2, tol), &issue_diag));
                    TLR_TRY(issue_diag());
                    Ctx::StatRead sr;
                    TLR_TRY(c.read_stats(jobs, sr));
                    // the side stream's diagonal Cholesky may still run: wait
                    // for the main stream alone unless the descriptor area
                    // must be recycled
                    if (c.desc_used > p->desc_bytes / 2)
                        TLR_TRY(c.sync_reset());
                    else
                        TLR_TRY(c.sync_main());
                    if (!jobs.empty() && *sr.status != 0) failed = true;
                    std::vector<int32_t> st(4 * jobs.size());
                    for (size_t q = 0; q < jobs.size(); ++q)
                        std::memcpy(&st[4 * q], &sr.raw[(size_t)(tile_index(jobs[q].i, jobs[q].j) - sr.t0) * 4],
                                    4 * sizeof(int32_t));
                    if (debug_enabled()) {
                        for (size_t q = 0; q < jobs.size(); ++q)
                            std::fprintf(stderr, "potrf col %d tile (%d,%d) R=%d k=%d r_old=%d write=%d num=%d flag=%d\n", j,
                                         jobs[q].i, jobs[q].j, Rj, jobs[q].k, jobs[q].r, st[4 * q], st[4 * q + 1],
                                         st[4 * q + 2]);
                    }
                    std::vector<Job> conv;
                    std::vector<CopyDesc> keep;
                    int64_t keep_max = 0;
                    for (size_t q = 0; q < jobs.size(); ++q) {
                        const Job &jb = jobs[q];
                        if (st[4 * q + 2]) {
                            kk[jb.i] = widen_k(p, jb.k, jb.kfull);
                            retry.push_back(jb.i);
                        } else if (p->dense_ok && st[4 * q + 1] > p->rcap) {
                            conv.push_back(jb);
                            r[(size_t)jb.i * nt + j] = nb;
                        } else {
                            const int rk = st[4 * q];
                            r[(size_t)jb.i * nt + j] = rk;
                            if (rk > 0 && !c.take_slot(jb.i, j, rk)) {
                                if (!failed) TLR_TRY(c.host_fail(TLR_ARENA_OVERFLOW, jb.i, j));
                                failed = true;
                            } else if (rk > 0) {
                                const int cv = p->mixed ? 2 : 0;
                                keep.push_back(CopyDesc{jb.Uout, c.U(jb.i, j), (int64_t)nb * rk, cv});
                                keep.push_back(CopyDesc{jb.Vout, c.V(jb.i, j), (int64_t)nb * rk, cv});
                                keep_max = std::max<int64_t>(keep_max, (int64_t)nb * rk);
                            }
                        }
                    }
                    if (!keep.empty()) {
                        TLR_PUSH(dkp, c, keep);
                        TLR_LAUNCH(c, copy_batched(dkp, (int)keep.size(), keep_max, s));
                    }
                    if (!conv.empty()) {  // over the cap: keep the Schur complement dense
                        TLR_TRY(schur_dense(conv));
                        std::vector<std::pair<int, int>> dt;
                        std::vector<const double *> ds;
                        for (const Job &jb : conv) {
                            dt.emplace_back(jb.i, jb.j);
                            ds.push_back(jb.D);
                        }
                        TLR_TRY(make_dense(c, dt, ds));
                    }
                    if (!conv.empty() || (p->dense_ok && !keep.empty())) TLR_TRY(c.sync_reset());
                }
                todo.swap(retry);
            }
            c.arena_used = mark;
        }
        TLR_TRY(issue_diag());
        if (failed) break;
        // the products below need the inverse from the side stream
        TLR_TRY(c.join());
        // L_ij = U_ij (L_jj^-1 V_ij)^T: T_i = L_jj^-1 V_ij into the arena (the
        // inverse comes from the side stream), then back into the tile's slot;
        // in groups that fit the arena, each group's copies queued before the
        // next group's products overwrite the scratch
        bool any_rank = false;
        {
            std::vector<GemmDesc> gi;
            std::vector<CopyDesc> back;
            int64_t mxw = 0;
            const size_t mark = c.arena_used;
            auto flush_group = [&]() -> tlr_status {
                if (gi.empty()) return TLR_OK;
                TLR_TRY(launch_gemms(c, false, false, gi, c.fb() | c.fc()));
                TLR_PUSH(dbk, c, back);
                TLR_LAUNCH(c, copy_batched(dbk, (int)back.size(), mxw, s));
                gi.clear();
                back.clear();
                mxw = 0;
                c.arena_used = mark;
                return TLR_OK;
            };
            for (int i : rows) {
                const int rij = r[(size_t)i * nt + j];
                if (rij <= 0) continue;
                any_rank = true;
                void *Ti = c.alloc_fac((size_t)nb * rij);
                if (!Ti) {
                    TLR_TRY(flush_group());
                    Ti = c.alloc_fac((size_t)nb * rij);
                    if (!Ti) return TLR_E_NOMEM;
                }
                gi.push_back(gd(c.linv(j), nb, c.V(i, j), nb, Ti, nb, nb, rij, nb, 1.0, 0.0));
                back.push_back(CopyDesc{Ti, c.V(i, j), (int64_t)nb * rij, p->mixed ? 2 : 0});
                mxw = std::max<int64_t>(mxw, (int64_t)nb * rij);
            }
            TLR_TRY(flush_group());
        }
        if (any_rank) {
            if (p->mixed) {
                // ||L_ij||_F = ||L_jj^-1 V_ij||_F for the noise of later Schur complements
                std::vector<NormDesc> nd;
                for (int i : rows)  // a tile of rank 0 gets norm 0
                    nd.push_back(NormDesc{static_cast<const float *>(c.V(i, j)), c.tstat(tile_index(i, j)),
                                          c.nrm_l() + (size_t)i * nt + j});
                TLR_PUSH(dnd, c, nd);
                TLR_LAUNCH(c, factor_norms(dnd, (int)nd.size(), nb, s));
            }
        }
        // no wait here: the next column's first launches queue behind these.
        // The descriptor area is recycled here, where the side stream has
        // finished (the main stream waited for it), once a quarter is used.
        if (c.desc_used > p->desc_bytes / 4) TLR_TRY(c.sync_reset());
    }
    TLR_TRY(c.sync_reset());
    TLR_TRY(c.store_dense());
    TLR_TRY(c.store_slots());
    TLR_HIP(hipMemcpyAsync(c.rL(), r.data(), sizeof(int32_t) * r.size(), hipMemcpyHostToDevice, s));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
}

// --------------------------------------------------------------- solve --

tlr_status solve_logdet(tlr_plan p, const double *d_z, void *d_ws, size_t ws_bytes, double *d_out, hipStream_t s) {
    if (!p || !d_z || !d_ws || !d_out) return TLR_E_INVAL;
    if (ws_bytes < p->off_fac) return TLR_E_NOMEM;
    Ctx c(p, d_ws, s);
    const int nt = p->nt, nb = p->nb;
    c.ws_size = ws_bytes;
    TLR_TRY(c.load_dense());
    TLR_TRY(c.load_slots());
    TLR_TRY(pad_copy(d_z, p->n, p->npad, c.yvec(), s));
    const size_t gb = gemv_desc_bytes();
    std::vector<char> hv(gb * std::max<int64_t>(p->ntiles, 1));
    std::vector<int> first(nt + 1, 0);
    size_t cnt = 0;
    for (int j = 0; j < nt; ++j) {
        first[j] = (int)cnt;
        for (int i = j + 1; i < nt; ++i) {
            make_gemv_desc(hv.data() + gb * cnt, c.U(i, j), c.V(i, j), c.ysol() + (int64_t)j * nb,
                           c.yvec() + (int64_t)i * nb, c.rL() + (size_t)i * nt + j);
            ++cnt;
        }
    }
    first[nt] = (int)cnt;
    char *dv = nullptr;
    if (cnt > 0) {
        dv = c.push(hv.data(), gb * cnt);
        if (!dv) return TLR_E_NOMEM;
    }
    for (int j = 0; j < nt; ++j) {
        // y_j = L_jj^-1 z_j (the inverse kept by the factorisation); then
        // z_i -= L_ij y_j below
        TLR_TRY(tri_gemv(c.linv(j), nb, c.yvec() + (int64_t)j * nb, c.ysol() + (int64_t)j * nb, c.params(), s));
        const int count = first[j + 1] - first[j];
        if (count > 0) TLR_LAUNCH(c, lr_gemv(dv + gb * first[j], count, nb, c.params(), s, p->mixed));
    }
    TLR_TRY(logdet_quad(c.diag(0), nb, nt, p->n, c.ysol(), c.params(), d_out, s));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
}

tlr_status status_read(tlr_plan p, const void *d_ws, tlr_devinfo *out, hipStream_t s) {
    if (!p || !d_ws || !out) return TLR_E_INVAL;
    Ctx c(p, const_cast<void *>(d_ws), s);
    ParamsBlock hb{};
    std::vector<int32_t> r((size_t)p->nt * p->nt, 0);
    TLR_HIP(hipStreamSynchronize(s));
    TLR_HIP(hipMemcpy(&hb, c.pblock(), sizeof(ParamsBlock), hipMemcpyDeviceToHost));
    TLR_HIP(hipMemcpy(r.data(), c.rL(), sizeof(int32_t) * r.size(), hipMemcpyDeviceToHost));
    out->code = hb.dp.status;
    out->tile_i = hb.dp.status ? hb.dp.fail_i : -1;
    out->tile_j = hb.dp.status ? hb.dp.fail_j : -1;
    int mx = 0;
    int64_t sum = 0;
    for (int i = 0; i < p->nt; ++i)
        for (int j = 0; j < i; ++j) {
            mx = std::max(mx, r[(size_t)i * p->nt + j]);
            sum += std::max(0, r[(size_t)i * p->nt + j]);
        }
    out->max_rank = mx;
    out->rank_sum = sum;
    return TLR_OK;
}

}  // namespace tlr

namespace tlr {
tlr_status ranks_read(tlr_plan p, const void *d_ws, int which, int32_t *d_out, hipStream_t s) {
    if (!p || !d_ws || !d_out || (which != 0 && which != 1)) return TLR_E_INVAL;
    Ctx c(p, const_cast<void *>(d_ws), s);
    const size_t cnt = (size_t)p->nt * p->nt;
    std::vector<int32_t> r(cnt);
    TLR_HIP(hipMemcpyAsync(r.data(), which == 0 ? c.rsig() : c.rL(), sizeof(int32_t) * cnt, hipMemcpyDeviceToHost, s));
    TLR_TRY(c.load_dense());  // synchronises
    for (size_t t = 0; t < cnt; ++t)
        if (c.dflag[t]) r[t] = -2;
    TLR_HIP(hipMemcpyAsync(d_out, r.data(), sizeof(int32_t) * cnt, hipMemcpyHostToDevice, s));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
}

void plan_shape(tlr_plan p, int64_t *n, int32_t *nb, int32_t *nt, int32_t *maxrank) {
    if (!p) return;
    if (n) *n = p->n;
    if (nb) *nb = p->nb;
    if (nt) *nt = p->nt;
    if (maxrank) *maxrank = p->rcap;
}
}  // namespace tlr

namespace tlr {
tlr_status tile_read(tlr_plan p, const void *d_ws, int i, int j, double *d_out, int32_t *h_rank, hipStream_t s) {
    if (!p || !d_ws || !d_out || i < 0 || j < 0 || i >= p->nt || j > i) return TLR_E_INVAL;
    Ctx c(p, const_cast<void *>(d_ws), s);
    const int nb = p->nb;
    TLR_TRY(c.load_dense());
    TLR_TRY(c.load_slots());
    if (i == j) {
        TLR_HIP(hipMemcpyAsync(d_out, c.diag(i), sizeof(double) * nb * nb, hipMemcpyDeviceToDevice, s));
        TLR_HIP(hipStreamSynchronize(s));
        if (h_rank) *h_rank = nb;
        return TLR_OK;
    }
    int32_t r = 0;
    TLR_HIP(hipMemcpyAsync(&r, c.rL() + (size_t)i * p->nt + j, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    TLR_HIP(hipStreamSynchronize(s));
    if (h_rank) *h_rank = r;
    std::vector<GemmDesc> g{gd(c.U(i, j), nb, c.V(i, j), nb, d_out, nb, nb, nb, std::max(r, 0), 1.0, 0.0)};
    TLR_TRY(launch_gemms(c, false, true, g, c.fa() | c.fb()));
    TLR_HIP(hipStreamSynchronize(s));
    return TLR_OK;
}
}  // namespace tlr
