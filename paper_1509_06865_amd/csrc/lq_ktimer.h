// Optional per-launch timing of one kernel class (instrumentation for the
// roofline measurement).  When a class is selected, every launcher of that
// class records a pair of HIP events on its own stream around the launch and
// adds the launch's algorithmic bytes; lq_kernel_timer_read sums the event
// intervals.  Off by default; then each hook is one integer compare.
#pragma once
#include <hip/hip_runtime.h>

namespace lq {

enum KernelClass { KT_WILSON = 0, KT_SAP = 1, KT_RESTRICT = 2, KT_PROLONG = 3, KT_COARSE = 4, KT_GRAM = 5,
                   KT_COMBINE = 6, KT_COUNT = 7 };

extern int g_ktimer_class;
void ktimer_begin(hipStream_t st);
void ktimer_end(hipStream_t st, double bytes);

// Records the launch(es) in its scope when class k is being timed.
struct KTimerScope {
  bool on;
  hipStream_t st;
  double bytes;
  KTimerScope(int k, hipStream_t s, double b) : on(g_ktimer_class == k), st(s), bytes(b) {
    if (on) ktimer_begin(st);
  }
  ~KTimerScope() {
    if (on) ktimer_end(st, bytes);
  }
};

}  // namespace lq
