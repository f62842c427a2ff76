// Batched evaluation of many independent problems (each its own n, tile
// size, locations, observations and theta) in one call.
//
// A batch plan holds one plan per problem and carves one caller workspace
// into their workspaces (256-byte aligned, in problem order).  An evaluation
// call runs the problems on W worker streams of default priority, W host
// threads taking problems widest first from a shared counter, so that the
// latency-bound factorisation of one problem overlaps the others' on the
// device.  Every worker stream first waits for the work already issued on the
// caller's stream; the caller's stream then waits for every worker stream.
// Results are bitwise those of one-at-a-time evaluations: every kernel is
// deterministic and the problems share no device memory.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "kernels.h"

namespace tlr {
tlr_status plan_create(tlr_plan *out, int64_t n, int nb, int maxrank, tlr_precision prec, uint32_t flags);
void plan_destroy(tlr_plan p);
size_t plan_ws_bytes(tlr_plan p);
tlr_status gen_tiles(tlr_plan p, const double *d_locs, tlr_theta th, void *d_ws, size_t ws_bytes, hipStream_t s);
tlr_status compress(tlr_plan p, double tol, void *d_ws, size_t ws_bytes, int32_t *d_ranks, hipStream_t s);
tlr_status potrf(tlr_plan p, void *d_ws, size_t ws_bytes, hipStream_t s);
tlr_status solve_logdet(tlr_plan p, const double *d_z, void *d_ws, size_t ws_bytes, double *d_out, hipStream_t s);
tlr_status status_read(tlr_plan p, const void *d_ws, tlr_devinfo *out, hipStream_t s);
}  // namespace tlr

struct tlr_batch_plan_s {
    std::vector<tlr_plan> plans;
    std::vector<size_t> offset;  // workspace offset of each problem
    std::vector<int64_t> n;
    size_t ws_bytes = 0;
};

namespace tlr {
namespace {

constexpr int kMaxBatchWorkers = 16;

// Worker streams (default priority), per device, created once and reused.
class StreamPool {
  public:
    bool get(int count, std::vector<hipStream_t> *out) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return false;
        std::lock_guard<std::mutex> g(mu_);
        auto &v = pool_[dev];
        while ((int)v.size() < count) {
            hipStream_t st = nullptr;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return false;
            note_stream_created();
            v.push_back(st);
        }
        out->assign(v.begin(), v.begin() + count);
        return true;
    }

  private:
    std::mutex mu_;
    std::vector<std::vector<hipStream_t>> pool_ = std::vector<std::vector<hipStream_t>>(64);
};

StreamPool &stream_pool() {
    static StreamPool *p = new StreamPool();  // never destroyed
    return *p;
}

// Batched calls on one device share its worker streams: one at a time.
std::mutex &batch_mutex() {
    static std::mutex *m = new std::mutex();
    return *m;
}

tlr_status eval_one(tlr_plan p, const double *locs, const double *z, tlr_theta th, double tol, void *ws,
                    size_t bytes, double *out, hipStream_t s) {
    TLR_TRY(gen_tiles(p, locs, th, ws, bytes, s));
    TLR_TRY(compress(p, tol, ws, bytes, nullptr, s));
    TLR_TRY(potrf(p, ws, bytes, s));
    return solve_logdet(p, z, ws, bytes, out, s);
}

}  // namespace

tlr_status batch_plan_create(tlr_batch_plan *out, int count, const int64_t *n, const int32_t *nb, int maxrank,
                             tlr_precision prec, uint32_t flags) {
    if (!out) return TLR_E_INVAL;
    *out = nullptr;
    if (count < 1 || !n || !nb) return TLR_E_INVAL;
    auto *bp = new tlr_batch_plan_s{};
    size_t off = 0;
    for (int p = 0; p < count; ++p) {
        tlr_plan pl = nullptr;
        const tlr_status st = plan_create(&pl, n[p], nb[p], maxrank, prec, flags);
        if (st != TLR_OK) {
            for (tlr_plan q : bp->plans) plan_destroy(q);
            delete bp;
            return st;
        }
        bp->plans.push_back(pl);
        bp->offset.push_back(off);
        bp->n.push_back(n[p]);
        off += align_up(plan_ws_bytes(pl), 256);
    }
    bp->ws_bytes = off;
    *out = bp;
    return TLR_OK;
}

void batch_plan_destroy(tlr_batch_plan bp) {
    if (!bp) return;
    for (tlr_plan q : bp->plans) plan_destroy(q);
    delete bp;
}

size_t batch_ws_bytes(tlr_batch_plan bp) { return bp ? bp->ws_bytes : 0; }

tlr_status loglik_batched(tlr_batch_plan bp, const double *const *locs, const double *const *z,
                          const tlr_theta *theta, double tol, void *d_ws, size_t ws_bytes, double *d_out,
                          int workers, hipStream_t s) {
    if (!bp || !locs || !z || !theta || !d_ws || !d_out) return TLR_E_INVAL;
    if (ws_bytes < bp->ws_bytes) return TLR_E_NOMEM;
    if (!(tol >= 0.0) || !std::isfinite(tol)) return TLR_E_INVAL;
    const int count = (int)bp->plans.size();
    for (int p = 0; p < count; ++p)
        if (!locs[p] || !z[p]) return TLR_E_INVAL;
    workers = std::max(1, std::min({workers, count, kMaxBatchWorkers}));
    std::lock_guard<std::mutex> serial(batch_mutex());
    std::vector<hipStream_t> ws;
    if (!stream_pool().get(workers, &ws)) return TLR_E_HIP;
    hipEvent_t ready = nullptr;
    TLR_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    tlr_status st0 = TLR_OK;
    if (hipEventRecord(ready, s) != hipSuccess) st0 = TLR_E_HIP;
    for (int w = 0; w < workers && st0 == TLR_OK; ++w)
        if (hipStreamWaitEvent(ws[w], ready, 0) != hipSuccess) st0 = TLR_E_HIP;
    if (st0 != TLR_OK) {
        (void)hipEventDestroy(ready);
        return st0;
    }
    // widest problems first: the longest evaluations start earliest
    std::vector<int> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return bp->n[a] > bp->n[b]; });
    std::atomic<int> next{0};
    std::vector<tlr_status> status(workers, TLR_OK);
    int dev = 0;
    (void)hipGetDevice(&dev);
    auto run = [&](int w) {
        (void)hipSetDevice(dev);
        for (;;) {
            const int k = next.fetch_add(1);
            if (k >= count) break;
            const int p = order[k];
            char *sub = static_cast<char *>(d_ws) + bp->offset[p];
            const tlr_status st = eval_one(bp->plans[p], locs[p], z[p], theta[p], tol, sub,
                                           plan_ws_bytes(bp->plans[p]), d_out + 3 * (size_t)p, ws[w]);
            if (st != TLR_OK && status[w] == TLR_OK) status[w] = st;
        }
    };
    std::vector<std::thread> threads;
    for (int w = 1; w < workers; ++w) threads.emplace_back(run, w);
    run(0);
    for (auto &t : threads) t.join();
    // the caller's stream waits for every worker stream
    tlr_status st = TLR_OK;
    for (int w = 0; w < workers; ++w) {
        if (status[w] != TLR_OK && st == TLR_OK) st = status[w];
        if (hipEventRecord(ready, ws[w]) != hipSuccess || hipStreamWaitEvent(s, ready, 0) != hipSuccess)
            st = TLR_E_HIP;
    }
    (void)hipEventDestroy(ready);
    return st;
}

tlr_status batch_status_read(tlr_batch_plan bp, const void *d_ws, int index, tlr_devinfo *out, hipStream_t s) {
    if (!bp || !d_ws || !out || index < 0 || index >= (int)bp->plans.size()) return TLR_E_INVAL;
    return status_read(bp->plans[index], static_cast<const char *>(d_ws) + bp->offset[index], out, s);
}

}  // namespace tlr
