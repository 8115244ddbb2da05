// Batched level-1 kernels: inner products with a fixed reduction tree (the
// result does not depend on timing, so reruns are bitwise identical), axpy
// against several basis vectors, scaling, precision and layout changes.
#include "lq_kernels.h"

namespace lq {
namespace {

constexpr int kDotThreads = 256;
constexpr int kDotChunks = 240;     // workgroups per (basis group, rhs) in stage 1
constexpr int kDotGroup = 8;        // basis vectors per workgroup

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Block-wide sum of a double; result valid in thread 0.  Fixed tree.
__device__ inline double block_sum(double v, double *lds) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) r += lds[w];
  return r;
}

// Stage 1: partial[row][k][chunk] for the rows g*G .. g*G + G - 1 of group g.
// Rows past nv read row nv - 1 and are dropped, so the loads carry no branches
// and stay in flight together; the launcher picks G (1, 2, 4, 8) as the
// smallest power of two covering nv, capped at kDotGroup, so few are wasted.
template <typename T, int G>
__global__ void __launch_bounds__(kDotThreads) k_dots_partial(int nv, const cplx<T> *__restrict__ vbase,
                                                              long long vstride, long long rstride,
                                                              const cplx<T> *__restrict__ w, long long wstride,
                                                              long long n, c128 *__restrict__ partial,
                                                              const int *__restrict__ active) {
  __shared__ double lds[kDotThreads / 64];
  const int chunk = blockIdx.x, k = blockIdx.y, grp = blockIdx.z;
  const int nchunks = gridDim.x, nrhs = gridDim.y;
  if (active && !active[k]) {
    if (threadIdx.x < G && grp * G + (int)threadIdx.x < nv)
      partial[((long long)(grp * G + threadIdx.x) * nrhs + k) * nchunks + chunk] = c128{0, 0};
    return;
  }
  const long long per = (n + nchunks - 1) / nchunks;
  const long long lo = chunk * per, hi = (lo + per < n) ? lo + per : n;
  const cplx<T> *wk = w + k * wstride;
  double re[G], im[G];
#pragma unroll
  for (int i = 0; i < G; ++i) { re[i] = 0; im[i] = 0; }
  const int i0 = grp * G;
  const cplx<T> *vk[G];
#pragma unroll
  for (int i = 0; i < G; ++i) vk[i] = vbase + (long long)(i0 + i < nv ? i0 + i : nv - 1) * vstride + k * rstride;
  for (long long e = lo + threadIdx.x; e < hi; e += kDotThreads) {
    const cplx<T> wv = wk[e];
#pragma unroll
    for (int i = 0; i < G; ++i) {
      const cplx<T> v = vk[i][e];
      re[i] += (double)v.re * wv.re + (double)v.im * wv.im;
      im[i] += (double)v.re * wv.im - (double)v.im * wv.re;
    }
  }
#pragma unroll
  for (int i = 0; i < G; ++i) {
    if (i0 + i >= nv) break;
    double sr = block_sum(re[i], lds);
    double si = block_sum(im[i], lds);
    if (threadIdx.x == 0) partial[((long long)(i0 + i) * nrhs + k) * nchunks + chunk] = c128{sr, si};
  }
}

// Stage 2: one wave per (i, k) sums the chunk partials in a fixed tree.
__global__ void k_dots_final(const c128 *__restrict__ partial, int nchunks, c128 *__restrict__ out) {
  const int ik = blockIdx.x;
  double re = 0, im = 0;
  for (int c = threadIdx.x; c < nchunks; c += 64) {
    re += partial[(long long)ik * nchunks + c].re;
    im += partial[(long long)ik * nchunks + c].im;
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (threadIdx.x == 0) out[ik] = c128{re, im};
}

template <typename T>
__global__ void k_multi_axpy(int nv, const cplx<T> *__restrict__ vbase, long long vstride, long long rstride,
                             const c128 *__restrict__ h, cplx<T> *__restrict__ w, long long wstride, long long n,
                             int nrhs, double sign, const int *__restrict__ active) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= n || (active && !active[k])) return;
  cplx<T> acc = w[k * wstride + e];
#pragma unroll 4
  for (int i = 0; i < nv; ++i) {
    const c128 hh = h[i * nrhs + k];
    const cplx<T> c = {(T)(sign * hh.re), (T)(sign * hh.im)};
    acc = acc + c * vbase[i * vstride + k * rstride + e];
  }
  w[k * wstride + e] = acc;
}

template <typename T>
__global__ void k_scale(const c128 *__restrict__ a, const cplx<T> *__restrict__ x, long long xstride,
                        cplx<T> *__restrict__ y, long long ystride, long long n, bool acc) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (e >= n) return;
  const cplx<T> c = {(T)a[k].re, (T)a[k].im};
  cplx<T> v = c * x[k * xstride + e];
  if (acc) v = v + y[k * ystride + e];
  y[k * ystride + e] = v;
}

template <typename To, typename Ti>
__global__ void k_convert(const cplx<Ti> *__restrict__ x, cplx<To> *__restrict__ y, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = cast<To>(x[e]);
}

// Canonical site index of blocked site s.
__device__ inline int canonical_of(const Geom &g, int s) {
  const SiteCoord c = decode(g, s);
  int x[4];
  for (int m = 0; m < 4; ++m) x[m] = c.a[m] * g.b[m] + c.l[m];
  return x[0] + g.L[0] * (x[1] + g.L[1] * (x[2] + g.L[2] * x[3]));
}

template <typename T>
__global__ void k_permute(Geom g, const cplx<T> *__restrict__ x, cplx<T> *__restrict__ y, bool to_blocked) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int f = blockIdx.y;
  const int n = canonical_of(g, s);
  const long long off = (long long)f * 12 * g.V;
  for (int i = 0; i < 12; ++i) {
    if (to_blocked) y[off + (long long)i * g.V + s] = x[off + (long long)i * g.V + n];
    else            y[off + (long long)i * g.V + n] = x[off + (long long)i * g.V + s];
  }
}

template <typename To>
__global__ void k_pack_links(Geom g, const c128 *__restrict__ U, cplx<To> *__restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int n = canonical_of(g, s);
  for (int i = 0; i < 36; ++i) out[(long long)i * g.V + s] = cast<To>(U[(long long)i * g.V + n]);
}

// ---- device-side bookkeeping of batched GMRES (one thread per system) ------
// State of system k: H column-major [(m+1) x m], Givens cosines cs[m] and sines
// sn[m], rotated right-hand side g[m+1], active flag, steps kk.

// Start of a restart cycle from nrm2[k] = ||r_k||^2: activity, g, 1/beta.
__global__ void k_arnoldi_start(int nrhs, int m, const c128 *__restrict__ nrm2, const double *__restrict__ bn,
                                double tol, c128 *__restrict__ g, int *__restrict__ active, int *__restrict__ kk,
                                c128 *__restrict__ coef) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const double beta = sqrt(fmax(nrm2[k].re, 0.0));
  const bool act = bn[k] > 0 && beta > tol * bn[k] && isfinite(beta);
  active[k] = act ? 1 : 0;
  kk[k] = 0;
  for (int i = 0; i <= m; ++i) g[(long long)k * (m + 1) + i] = c128{0, 0};
  g[(long long)k * (m + 1)] = c128{act ? beta : 0.0, 0};
  coef[k] = c128{act ? 1.0 / beta : 0.0, 0};
}

// Step j: column h = h1 + h2 (CGS twice) with subdiagonal sqrt(nrm2), Givens
// update, convergence test, and the normalisation factor of the new vector.
__global__ void k_arnoldi_update(int j, int m, int nrhs, const c128 *__restrict__ h1, const c128 *__restrict__ h2,
                                 const c128 *__restrict__ nrm2, c128 *__restrict__ H, double *__restrict__ cs,
                                 c128 *__restrict__ sn, c128 *__restrict__ g, const double *__restrict__ bn, double tol,
                                 int *__restrict__ active, int *__restrict__ kk, c128 *__restrict__ coef,
                                 int *__restrict__ bad) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  if (!active[k]) { coef[k] = c128{0, 0}; return; }
  c128 *Hk = H + (long long)k * (m + 1) * m + (long long)j * (m + 1);
  double *ck = cs + (long long)k * m;
  c128 *sk = sn + (long long)k * m;
  c128 *gk = g + (long long)k * (m + 1);
  for (int i = 0; i <= j; ++i) Hk[i] = h1[i * nrhs + k] + h2[i * nrhs + k];
  const double hn = sqrt(fmax(nrm2[k].re, 0.0));
  Hk[j + 1] = c128{hn, 0};
  for (int i = 0; i < j; ++i) {
    const c128 a = Hk[i], b = Hk[i + 1];
    Hk[i] = ck[i] * a + sk[i] * b;
    Hk[i + 1] = (-1.0) * (conj(sk[i]) * a) + ck[i] * b;
  }
  const c128 a = Hk[j], b = Hk[j + 1];
  const double na = sqrt(norm2(a));
  double c;
  c128 s;
  if (na == 0.0) { c = 0; s = c128{1, 0}; }
  else {
    const double r = sqrt(norm2(a) + norm2(b));
    c = na / r;
    s = (1.0 / (na * r)) * (a * conj(b));
  }
  ck[j] = c; sk[j] = s;
  Hk[j] = c * a + s * b;
  Hk[j + 1] = c128{0, 0};
  gk[j + 1] = (-1.0) * (conj(s) * gk[j]);
  gk[j] = c * gk[j];
  const double res = sqrt(norm2(gk[j + 1]));
  kk[k] = j + 1;
  if (!isfinite(hn) || !isfinite(res)) { *bad = 1; active[k] = 0; coef[k] = c128{0, 0}; return; }
  if (res <= tol * bn[k] || hn == 0.0 || j + 1 >= m) active[k] = 0;
  coef[k] = c128{active[k] ? 1.0 / hn : 0.0, 0};
}

// Back substitution R y = g for each system; Y [m][nrhs], zero beyond kk[k].
__global__ void k_arnoldi_solve(int m, int nrhs, const c128 *__restrict__ H, const c128 *__restrict__ g,
                                const int *__restrict__ kk, c128 *__restrict__ Y) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const c128 *Hk = H + (long long)k * (m + 1) * m;
  const c128 *gk = g + (long long)k * (m + 1);
  const int n = kk[k];
  for (int i = m - 1; i >= n; --i) Y[i * nrhs + k] = c128{0, 0};
  for (int i = n - 1; i >= 0; --i) {
    c128 v = gk[i];
    for (int l = i + 1; l < n; ++l) v = v - Hk[(long long)l * (m + 1) + i] * Y[l * nrhs + k];
    const c128 d = Hk[(long long)i * (m + 1) + i];
    const double dd = norm2(d);
    Y[i * nrhs + k] = (1.0 / dd) * (v * conj(d));
  }
}

}  // namespace

void launch_arnoldi_start(int nrhs, int m, const c128 *nrm2, const double *bn, double tol, c128 *g, int *active,
                          int *kk, c128 *coef, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_start, dim3(1), dim3(64), 0, st, nrhs, m, nrm2, bn, tol, g, active, kk, coef);
  LQ_HIP(hipGetLastError());
}
void launch_arnoldi_update(int j, int m, int nrhs, const c128 *h1, const c128 *h2, const c128 *nrm2, c128 *H,
                           double *cs, c128 *sn, c128 *g, const double *bn, double tol, int *active, int *kk,
                           c128 *coef, int *bad, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_update, dim3(1), dim3(64), 0, st, j, m, nrhs, h1, h2, nrm2, H, cs, sn, g, bn, tol,
                     active, kk, coef, bad);
  LQ_HIP(hipGetLastError());
}
void launch_arnoldi_solve(int m, int nrhs, const c128 *H, const c128 *g, const int *kk, c128 *Y, hipStream_t st) {
  hipLaunchKernelGGL(k_arnoldi_solve, dim3(1), dim3(64), 0, st, m, nrhs, H, g, kk, Y);
  LQ_HIP(hipGetLastError());
}

size_t dots_scratch_elems(int nv, int nrhs) {
  const int groups = (nv + kDotGroup - 1) / kDotGroup;
  return (size_t)groups * kDotGroup * nrhs * kDotChunks;
}

template <typename T>
void launch_dots(int nv, const cplx<T> *vbase, long long vstride, long long rstride, const cplx<T> *w,
                 long long wstride, long long n, int nrhs, c128 *out, c128 *scratch, hipStream_t st,
                 const int *active) {
  if (nv <= 0) return;
  int nchunks = (int)((n + 4 * kDotThreads - 1) / (4 * kDotThreads));
  if (nchunks > kDotChunks) nchunks = kDotChunks;
  if (nchunks < 1) nchunks = 1;
  c128 *partial = scratch;
  const int G = (nv > 4) ? kDotGroup : (nv > 2) ? 4 : nv;      // 1, 2, 4 or 8
  const dim3 grid(nchunks, nrhs, (nv + G - 1) / G);
  switch (G) {
    case 1:
      hipLaunchKernelGGL((k_dots_partial<T, 1>), grid, dim3(kDotThreads), 0, st, nv, vbase, vstride, rstride, w,
                         wstride, n, partial, active);
      break;
    case 2:
      hipLaunchKernelGGL((k_dots_partial<T, 2>), grid, dim3(kDotThreads), 0, st, nv, vbase, vstride, rstride, w,
                         wstride, n, partial, active);
      break;
    case 4:
      hipLaunchKernelGGL((k_dots_partial<T, 4>), grid, dim3(kDotThreads), 0, st, nv, vbase, vstride, rstride, w,
                         wstride, n, partial, active);
      break;
    default:
      hipLaunchKernelGGL((k_dots_partial<T, kDotGroup>), grid, dim3(kDotThreads), 0, st, nv, vbase, vstride,
                         rstride, w, wstride, n, partial, active);
  }
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_dots_final, dim3(nv * nrhs), dim3(64), 0, st, partial, nchunks, out);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_multi_axpy(int nv, const cplx<T> *vbase, long long vstride, long long rstride, const c128 *h,
                       cplx<T> *w, long long wstride, long long n, int nrhs, double sign, hipStream_t st,
                       const int *active) {
  if (nv <= 0) return;
  hipLaunchKernelGGL((k_multi_axpy<T>), dim3(blocks_for(n, 256), nrhs), dim3(256), 0, st, nv, vbase, vstride,
                     rstride, h, w, wstride, n, nrhs, sign, active);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_scale(const c128 *a, const cplx<T> *x, long long xstride, cplx<T> *y, long long ystride,
                  long long n, int nrhs, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL((k_scale<T>), dim3(blocks_for(n, 256), nrhs), dim3(256), 0, st, a, x, xstride, y, ystride,
                     n, accumulate);
  LQ_HIP(hipGetLastError());
}

template <typename To, typename Ti>
void launch_convert(const cplx<Ti> *x, cplx<To> *y, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_convert<To, Ti>), dim3(blocks_for(n, 256)), dim3(256), 0, st, x, y, n);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_permute(const Geom &g, const cplx<T> *x, cplx<T> *y, int nf, bool to_blocked, hipStream_t st) {
  hipLaunchKernelGGL((k_permute<T>), dim3(blocks_for(g.V, 256), nf), dim3(256), 0, st, g, x, y, to_blocked);
  LQ_HIP(hipGetLastError());
}

template <typename To>
void launch_pack_links(const Geom &g, const c128 *U, cplx<To> *out, hipStream_t st) {
  hipLaunchKernelGGL((k_pack_links<To>), dim3(blocks_for(g.V, 256)), dim3(256), 0, st, g, U, out);
  LQ_HIP(hipGetLastError());
}

#define LQ_INST(T)                                                                                         \
  template void launch_dots<T>(int, const cplx<T> *, long long, long long, const cplx<T> *, long long,      \
                               long long, int, c128 *, c128 *, hipStream_t, const int *);                 \
  template void launch_multi_axpy<T>(int, const cplx<T> *, long long, long long, const c128 *, cplx<T> *,   \
                                     long long, long long, int, double, hipStream_t, const int *);        \
  template void launch_scale<T>(const c128 *, const cplx<T> *, long long, cplx<T> *, long long, long long, \
                                int, bool, hipStream_t);                                                  \
  template void launch_permute<T>(const Geom &, const cplx<T> *, cplx<T> *, int, bool, hipStream_t);        \
  template void launch_pack_links<T>(const Geom &, const c128 *, cplx<T> *, hipStream_t);
LQ_INST(float)
LQ_INST(double)
#undef LQ_INST
template void launch_convert<float, double>(const c128 *, c64 *, long long, hipStream_t);
template void launch_convert<double, float>(const c64 *, c128 *, long long, hipStream_t);
template void launch_convert<double, double>(const c128 *, c128 *, long long, hipStream_t);
template void launch_convert<float, float>(const c64 *, c64 *, long long, hipStream_t);

}  // namespace lq
