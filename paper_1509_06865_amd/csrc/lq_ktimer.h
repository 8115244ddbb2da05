// Optional per-launch timing of one kernel class (instrumentation for the
// roofline measurement).  When a class is selected, its launchers take a pair
// of HIP events from a pool and launch through hipExtLaunchKernelGGL, which
// records the events in the kernel's own dispatch packet (so the interval is
// the kernel's execution, without launch gaps), and add the launch's
// algorithmic bytes; lq_kernel_timer_read sums the intervals.  Off by
// default; then each hook is one integer compare.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

namespace lq {

enum KernelClass { KT_WILSON = 0, KT_SAP = 1, KT_RESTRICT = 2, KT_PROLONG = 3, KT_COARSE = 4, KT_GRAM = 5,
                   KT_COMBINE = 6, KT_COUNT = 7 };

extern int g_ktimer_class;
// a pair of unrecorded events for the next launch and its bytes; false if the
// pool cannot grow (then the launch runs untimed)
bool ktimer_acquire(hipEvent_t *start, hipEvent_t *stop, double bytes);

struct KTimerScope {
  bool on = false;
  hipEvent_t a = nullptr, b = nullptr;
  KTimerScope(int k, double bytes) {
    if (g_ktimer_class == k) on = ktimer_acquire(&a, &b, bytes);
  }
};

}  // namespace lq

// Launch `kernel`, timed through the dispatch packet when the scope is on.
#define LQ_LAUNCH(kt, kernel, grid, block, shmem, st, ...)                                         \
  do {                                                                                             \
    if ((kt).on)                                                                                   \
      hipExtLaunchKernelGGL(kernel, grid, block, shmem, st, (kt).a, (kt).b, 0, __VA_ARGS__);       \
    else                                                                                           \
      hipLaunchKernelGGL(kernel, grid, block, shmem, st, __VA_ARGS__);                             \
  } while (0)
