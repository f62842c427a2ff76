// Opt-in per-kernel launch timer.
//
// When enabled, every instrumented launch is bracketed by two HIP events
// recorded on the stream the kernel is launched on, so the elapsed time
// between them is that launch's duration on the device.  Each launch also
// carries its algorithmic work as counted on the host: the floating-point
// operations the method needs and the bytes it must move to or from HBM
// (each operand read once, each result written once).  A launch whose sizes
// are only known on the device (a rank computed by an earlier kernel) is
// marked inexact: its time is recorded but its work is not counted.
//
// Statistics are kept per kernel function, so a class matches one symbol in
// a profiler's kernel trace.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace tlr {

int ktimer_class(const char *name);  // stable id of a kernel class
bool ktimer_on();
void ktimer_poll();  // fold finished launches into the totals (never waits)

struct KStat {
    char name[48];
    int64_t launches;
    double total_ms;
    int64_t exact_launches;
    double exact_ms;
    double flops;
    double bytes;
};
void ktimer_enable(bool on);
void ktimer_select(int cls);  // time only this class (-1: every class)
void ktimer_reset();
int ktimer_read(KStat *out, int max);  // waits for every pending launch

class KTimer {
  public:
    KTimer(int cls, hipStream_t s, double flops, double bytes, bool exact = true);
    ~KTimer();
    KTimer(const KTimer &) = delete;
    KTimer &operator=(const KTimer &) = delete;

  private:
    int cls_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr;
    double flops_, bytes_;
    bool exact_;
};

}  // namespace tlr
