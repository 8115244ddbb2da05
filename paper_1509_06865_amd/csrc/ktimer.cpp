// Event pool and totals of the kernel-class timer (lq_ktimer.h).
#include "lq_ktimer.h"
#include "lqmg.h"

#include <vector>

namespace lq {

int g_ktimer_class = -1;

namespace {
struct Pool {
  std::vector<hipEvent_t> a, b;
  std::vector<double> bytes;
  size_t used = 0;
};
Pool &pool() {
  static Pool p;
  return p;
}
}  // namespace

bool ktimer_acquire(hipEvent_t *start, hipEvent_t *stop, double bytes) {
  Pool &p = pool();
  if (p.used == p.a.size()) {
    hipEvent_t x, y;
    if (hipEventCreate(&x) != hipSuccess) { (void)hipGetLastError(); return false; }
    if (hipEventCreate(&y) != hipSuccess) { (void)hipGetLastError(); (void)hipEventDestroy(x); return false; }
    p.a.push_back(x);
    p.b.push_back(y);
    p.bytes.push_back(0.0);
  }
  *start = p.a[p.used];
  *stop = p.b[p.used];
  p.bytes[p.used] = bytes;
  ++p.used;
  return true;
}

}  // namespace lq

extern "C" int lq_kernel_timer_start(int kind) {
  if (kind < -1 || kind >= lq::KT_COUNT) return LQ_ERR_ARG;
  lq::pool().used = 0;
  lq::g_ktimer_class = kind;
  return LQ_OK;
}

extern "C" int lq_kernel_timer_read(long long *launches, double *ms_total, double *bytes_total) {
  lq::Pool &p = lq::pool();
  double ms = 0, by = 0;
  for (size_t i = 0; i < p.used; ++i) {
    if (hipEventSynchronize(p.b[i]) != hipSuccess) return LQ_ERR_HIP;
    float e = 0;
    if (hipEventElapsedTime(&e, p.a[i], p.b[i]) != hipSuccess) return LQ_ERR_HIP;
    ms += e;
    by += p.bytes[i];
  }
  if (launches) *launches = (long long)p.used;
  if (ms_total) *ms_total = ms;
  if (bytes_total) *bytes_total = by;
  return LQ_OK;
}
