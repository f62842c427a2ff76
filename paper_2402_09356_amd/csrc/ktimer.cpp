#include "ktimer.h"

#include <atomic>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

namespace tlr {
namespace {

struct Pending {
    int cls;
    int dev;
    hipEvent_t a, b;
    double flops, bytes;
    bool exact;
};

struct State {
    std::mutex mu;
    std::atomic<bool> on{false};
    std::atomic<int> sel{-1};  // the one class timed, or -1 for all
    std::vector<std::string> names;
    std::vector<KStat> stats;
    std::deque<Pending> pending;
    std::map<int, std::vector<hipEvent_t>> pool;  // per device
};

State &st() {
    static State *s = new State();  // never destroyed: events may outlive static teardown
    return *s;
}

hipEvent_t get_event(State &S, int dev) {
    auto &v = S.pool[dev];
    if (!v.empty()) {
        hipEvent_t e = v.back();
        v.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Fold the finished launches at the front of the queue; with `block`, wait
// for all of them.  Caller holds the mutex.
void harvest(State &S, bool block) {
    while (!S.pending.empty()) {
        Pending &p = S.pending.front();
        if (!block && hipEventQuery(p.b) == hipErrorNotReady) break;
        (void)hipEventSynchronize(p.b);
        float ms = 0.0f;
        if (hipEventElapsedTime(&ms, p.a, p.b) != hipSuccess) ms = 0.0f;
        KStat &k = S.stats[p.cls];
        k.launches += 1;
        k.total_ms += ms;
        if (p.exact) {
            k.exact_launches += 1;
            k.exact_ms += ms;
            k.flops += p.flops;
            k.bytes += p.bytes;
        }
        S.pool[p.dev].push_back(p.a);
        S.pool[p.dev].push_back(p.b);
        S.pending.pop_front();
    }
}

}  // namespace

int ktimer_class(const char *name) {
    State &S = st();
    std::lock_guard<std::mutex> g(S.mu);
    for (size_t i = 0; i < S.names.size(); ++i)
        if (S.names[i] == name) return (int)i;
    S.names.emplace_back(name);
    KStat k{};
    std::strncpy(k.name, name, sizeof(k.name) - 1);
    S.stats.push_back(k);
    return (int)S.names.size() - 1;
}

bool ktimer_on() { return st().on.load(std::memory_order_relaxed); }

void ktimer_enable(bool on) { st().on.store(on); }

void ktimer_select(int cls) { st().sel.store(cls); }

void ktimer_poll() {
    State &S = st();
    if (!S.on.load(std::memory_order_relaxed)) return;
    std::lock_guard<std::mutex> g(S.mu);
    harvest(S, false);
}

void ktimer_reset() {
    State &S = st();
    std::lock_guard<std::mutex> g(S.mu);
    harvest(S, true);
    for (auto &k : S.stats) {
        KStat z{};
        std::memcpy(z.name, k.name, sizeof(z.name));
        k = z;
    }
}

int ktimer_read(KStat *out, int max) {
    State &S = st();
    std::lock_guard<std::mutex> g(S.mu);
    harvest(S, true);
    const int n = (int)S.stats.size();
    for (int i = 0; i < n && i < max; ++i) out[i] = S.stats[i];
    return n;
}

KTimer::KTimer(int cls, hipStream_t s, double flops, double bytes, bool exact)
    : cls_(cls), s_(s), flops_(flops), bytes_(bytes), exact_(exact) {
    if (!ktimer_on()) return;
    State &S = st();
    const int sel = S.sel.load(std::memory_order_relaxed);
    if (sel >= 0 && sel != cls) return;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(S.mu);
    a_ = get_event(S, dev);
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) {
        S.pool[dev].push_back(a_);
        a_ = nullptr;
    }
}

KTimer::~KTimer() {
    if (!a_) return;
    State &S = st();
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> g(S.mu);
    hipEvent_t b = get_event(S, dev);
    if (!b || hipEventRecord(b, s_) != hipSuccess) {
        S.pool[dev].push_back(a_);
        if (b) S.pool[dev].push_back(b);
        return;
    }
    S.pending.push_back(Pending{cls_, dev, a_, b, flops_, bytes_, exact_});
}

}  // namespace tlr
