// Wilson-Dirac stencil for Q = gamma5 D (sec. 2), one thread per lattice site.
//
// Each hop is applied in spin-projected form (lq_dslash.h): only the two-spin
// upper half of (1 -+ gamma_mu) psi is multiplied by the link.
#include "lq_kernels.h"
#include "lq_dslash.h"

namespace lq {
namespace {

// One thread per site and R right-hand sides: each link is loaded once and
// applied to the R fields, so the links are read once per group of R fields.
// With CLOV the site term carries the clover term C(x) (lq_dslash.h).
template <typename T, int MODE, int R, bool CLOV>
__global__ void __launch_bounds__(256) k_wilson(Geom g, const cplx<T> *__restrict__ U,
                                                const cplx<T> *__restrict__ xin, cplx<T> *__restrict__ yout,
                                                const cplx<T> *__restrict__ bin, T m0, Shifts sig, int nrhs,
                                                const cplx<T> *__restrict__ C) {
  const int s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int k0 = blockIdx.y * R;
  const int nr = (nrhs - k0 < R) ? nrhs - k0 : R;      // same for the whole launch row
  const long long fs = 12LL * g.V;
  const cplx<T> *x = xin + k0 * fs;
  const SiteCoord c = decode(g, s);
  cplx<T> acc[R][12], p[12], m[9];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[r][i] = mk<T>(0, 0);
  // a rolled loop over directions bounds the live ranges (one hop pair at a time)
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    float sg;
    bool in;
    const int sf = neighbour(g, s, c, mu, true, &sg, &in);
    load_link(U, g.V, mu, s, m);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= nr) break;
      load_spinor(x + r * fs, g.V, sf, p);
      hop_link(mu, true, p, m, (T)sg, acc[r]);
    }
    const int sb = neighbour(g, s, c, mu, false, &sg, &in);
    load_link(U, g.V, mu, sb, m);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (r >= nr) break;
      load_spinor(x + r * fs, g.V, sb, p);
      hop_link(mu, false, p, m, (T)sg, acc[r]);
    }
  }
  const T diag = (T)4 + m0;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= nr) break;
    const long long off = (k0 + r) * fs;
    load_spinor(x + r * fs, g.V, s, p);
    if constexpr (CLOV) clover_add(C, g.V, s, p, (T)-2, acc[r]);     // -1/2 acc then adds C p
    const T sgm = (T)sig.s[k0 + r];
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cplx<T> d = diag * p[i] - (T)0.5 * acc[r][i];
      if (i >= 6) d = -d;                        // gamma5
      d = d - sgm * p[i];
      if (MODE == W_RESID) d = bin[off + (long long)i * g.V + s] - d;
      yout[off + (long long)i * g.V + s] = d;
    }
  }
}

// Canonical layout (one block), one field: each thread walks a column of up
// to TC timeslices at one spatial site.  The forward t neighbour it loads is
// the next site's own spinor, and the backward t hop into the next site,
// (1 + gamma_t) U_t(n)^dag x(n), is formed from the link and spinor already in
// registers and carried as a projected half spinor, so every spinor and t link
// is read once per column.  Consecutive threads take consecutive spatial
// sites (coalesced); column chunks are renumbered per XCD like the other
// stencil launches.
template <typename T, bool CLOV>
__global__ void __launch_bounds__(256) k_wilson_tcol(Geom g, const cplx<T> *__restrict__ U,
                                                     const cplx<T> *__restrict__ x, cplx<T> *__restrict__ y, T m0,
                                                     int TC, const cplx<T> *__restrict__ C) {
  const int L0 = g.L[0], L1 = g.L[1], L2 = g.L[2], L3 = g.L[3];
  const int S3 = L0 * L1 * L2;
  const int nchunk = (L3 + TC - 1) / TC;
  const int col = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (col >= S3 * nchunk) return;
  const int chunk = col / S3;
  const int sp = col - chunk * S3;
  const int t0 = chunk * TC, t1 = (t0 + TC < L3) ? t0 + TC : L3;
  const long long V = g.V;
  const int cx = sp % L0, cy = (sp / L0) % L1, cz = sp / (L0 * L1);
  // spatial neighbours (periodic) of the column, forward and backward
  int nf[3], nb[3];
  nf[0] = (cx + 1 < L0) ? sp + 1 : sp - (L0 - 1);
  nb[0] = (cx > 0) ? sp - 1 : sp + (L0 - 1);
  nf[1] = (cy + 1 < L1) ? sp + L0 : sp - (L1 - 1) * L0;
  nb[1] = (cy > 0) ? sp - L0 : sp + (L1 - 1) * L0;
  nf[2] = (cz + 1 < L2) ? sp + L0 * L1 : sp - (L2 - 1) * L0 * L1;
  nb[2] = (cz > 0) ? sp - L0 * L1 : sp + (L2 - 1) * L0 * L1;
  const T tsign = (T)g.tbc;
  cplx<T> xc[12], p[12], m[9], acc[12];
  Half2<T> h, ub;
  // backward t hop into t0, from t0 - 1 (boundary sign when t0 = 0)
  {
    const int tm = (t0 > 0) ? t0 - 1 : L3 - 1;
    const int n = sp + tm * S3;
    load_spinor(x, V, n, p);
    load_link(U, V, 3, n, m);
    project(3, (T)1, p, h);
    link_mul(m, h, ub, true);
  }
  T ubsign = (t0 > 0) ? (T)1 : tsign;
  load_spinor(x, V, sp + t0 * S3, xc);
  const T diag = (T)4 + m0;
  for (int t = t0; t < t1; ++t) {
    const int n = sp + t * S3;
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
    reconstruct(3, (T)1, ub, ubsign, acc);
    // spatial hops
#pragma unroll 1
    for (int mu = 0; mu < 3; ++mu) {
      const int f = nf[mu] + t * S3, b = nb[mu] + t * S3;
      load_spinor(x, V, f, p);
      load_link(U, V, mu, n, m);
      hop_link(mu, true, p, m, (T)1, acc);
      load_spinor(x, V, b, p);
      load_link(U, V, mu, b, m);
      hop_link(mu, false, p, m, (T)1, acc);
    }
    // forward t hop; its spinor is the next site's own
    const bool wrap = (t + 1 == L3);
    load_spinor(x, V, wrap ? sp : n + S3, p);
    load_link(U, V, 3, n, m);
    hop_link(3, true, p, m, wrap ? tsign : (T)1, acc);
    // backward t hop into t + 1, carried
    project(3, (T)1, xc, h);
    link_mul(m, h, ub, true);
    ubsign = (T)1;
    if constexpr (CLOV) clover_add(C, V, n, xc, (T)-2, acc);
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      cplx<T> d = diag * xc[i] - (T)0.5 * acc[i];
      if (i >= 6) d = -d;                        // gamma5
      y[(long long)i * V + n] = d;
      xc[i] = p[i];
    }
  }
}

// Parts of Q for the Galerkin product, per column field j.
template <typename T, bool CLOV>
__global__ void __launch_bounds__(256) k_coarse_parts(Geom g, const cplx<T> *__restrict__ U,
                                                      const cplx<T> *__restrict__ xin, long long xstride,
                                                      cplx<T> *__restrict__ parts, T m0, const int *half_dev,
                                                      const cplx<T> *__restrict__ C) {
  const int s = xcd_tile(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const int j = blockIdx.y;
  const int half = half_dev[j];
  const cplx<T> *x = xin + (long long)j * xstride;
  cplx<T> *out = parts + (long long)j * 5 * 12 * g.V;
  const SiteCoord c = decode(g, s);
  // x with the unused gamma5 half read as zero
  auto ld = [&](int site, cplx<T> p[12]) {
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const bool use = (half == 0) ? (i < 6) : (i >= 6);
      p[i] = use ? x[(long long)i * g.V + site] : mk<T>(0, 0);
    }
  };
  cplx<T> self[12], cross[12], p[12];
  ld(s, p);
#pragma unroll
  for (int i = 0; i < 12; ++i) self[i] = ((T)4 + m0) * p[i];
  if constexpr (CLOV) clover_add(C, g.V, s, p, (T)1, self);         // keeps the gamma5 half
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    float sg;
    bool in;
    const int sf = neighbour(g, s, c, mu, true, &sg, &in);
    ld(sf, p);
#pragma unroll
    for (int i = 0; i < 12; ++i) cross[i] = mk<T>(0, 0);
    hop(mu, true, p, U, g.V, s, (T)sg, cross);
    if (in) {
#pragma unroll
      for (int i = 0; i < 12; ++i) { self[i] = self[i] - (T)0.5 * cross[i]; cross[i] = mk<T>(0, 0); }
    }
    // crossing part, -1/2 and gamma5 applied
#pragma unroll
    for (int i = 0; i < 12; ++i)
      out[(long long)((1 + mu) * 12 + i) * g.V + s] = (i >= 6 ? (T)0.5 : (T)-0.5) * cross[i];
    const int sb = neighbour(g, s, c, mu, false, &sg, &in);
    if (in) {
      ld(sb, p);
#pragma unroll
      for (int i = 0; i < 12; ++i) cross[i] = mk<T>(0, 0);
      hop(mu, false, p, U, g.V, sb, (T)sg, cross);
#pragma unroll
      for (int i = 0; i < 12; ++i) self[i] = self[i] - (T)0.5 * cross[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 12; ++i) out[(long long)i * g.V + s] = (i >= 6) ? -self[i] : self[i];
}

// fields per thread in the Wilson kernel: registers allow 2 in FP64, 4 in FP32
template <typename T> constexpr int wilson_group() { return sizeof(T) == 4 ? 4 : 2; }

template <typename T, bool CLOV>
void wilson_launch(KTimerScope &kt, const Geom &g, const cplx<T> *U, const cplx<T> *x, cplx<T> *y,
                   const cplx<T> *b, double m0, const Shifts &sig, int nrhs, int mode, hipStream_t st,
                   const cplx<T> *C) {
  constexpr int R = wilson_group<T>();
  // Column kernel: the timeslices per thread are chosen for about one workgroup
  // of 256 columns per CU (32^3 x 64: two columns of 32 timeslices per spatial
  // site, 256 workgroups).  Fewer, longer columns keep the timeslices that each
  // XCD reads at one time within its L2; measured at 32^3 x 64 in FP64, 32
  // timeslices per column took 0.46 ms against 0.53 (16) and 0.545 (8).
  const long long S3 = (long long)g.L[0] * g.L[1] * g.L[2];
  const long long want = (256LL * 256 + S3 / 2) / S3;
  const int nchunk = (int)(want < 1 ? 1 : (want > g.L[3] ? g.L[3] : want));
  const int TC = (g.L[3] + nchunk - 1) / nchunk;
  const long long cols = S3 * ((g.L[3] + TC - 1) / TC);
  // used when the columns fill the GPU and are at least 4 timeslices long
  if (nrhs == 1 && mode == W_QSHIFT && g.nblk == 1 && sig.s[0] == 0.0 && TC >= 4 && cols >= 192 * 256) {
    LQ_LAUNCH(kt, (k_wilson_tcol<T, CLOV>), dim3(blocks_for(cols, 256)), dim3(256), 0, st, g, U, x, y, (T)m0, TC,
              C);
  } else if (nrhs == 1) {
    const dim3 grid(blocks_for(g.V, 256), 1);
    if (mode == W_QSHIFT)
      LQ_LAUNCH(kt, (k_wilson<T, W_QSHIFT, 1, CLOV>), grid, dim3(256), 0, st, g, U, x, y, b, (T)m0, sig, nrhs, C);
    else
      LQ_LAUNCH(kt, (k_wilson<T, W_RESID, 1, CLOV>), grid, dim3(256), 0, st, g, U, x, y, b, (T)m0, sig, nrhs, C);
  } else {
    const dim3 grid(blocks_for(g.V, 256), (nrhs + R - 1) / R);
    if (mode == W_QSHIFT)
      LQ_LAUNCH(kt, (k_wilson<T, W_QSHIFT, R, CLOV>), grid, dim3(256), 0, st, g, U, x, y, b, (T)m0, sig, nrhs, C);
    else
      LQ_LAUNCH(kt, (k_wilson<T, W_RESID, R, CLOV>), grid, dim3(256), 0, st, g, U, x, y, b, (T)m0, sig, nrhs, C);
  }
}

}  // namespace

template <typename T>
void launch_wilson(const Geom &g, const cplx<T> *U, const cplx<T> *x, cplx<T> *y, const cplx<T> *b,
                   double m0, const Shifts &sig, int nrhs, int mode, hipStream_t st, const cplx<T> *C) {
  if (nrhs <= 0) return;
  // algorithmic bytes: links once, each field in and out (and b when forming
  // residuals), the clover blocks once
  KTimerScope kt(KT_WILSON, (double)g.V * (36.0 + (C ? 42.0 : 0.0) + nrhs * (mode == W_RESID ? 36.0 : 24.0)) *
                                sizeof(cplx<T>));
  if (C) wilson_launch<T, true>(kt, g, U, x, y, b, m0, sig, nrhs, mode, st, C);
  else wilson_launch<T, false>(kt, g, U, x, y, b, m0, sig, nrhs, mode, st, C);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_coarse_parts(const Geom &g, const cplx<T> *U, const cplx<T> *x, const int *half_dev,
                         int nf, long long xstride, cplx<T> *parts, double m0, hipStream_t st, const cplx<T> *C) {
  dim3 grid(blocks_for(g.V, 256), nf);
  if (C)
    hipLaunchKernelGGL((k_coarse_parts<T, true>), grid, dim3(256), 0, st, g, U, x, xstride, parts, (T)m0,
                       half_dev, C);
  else
    hipLaunchKernelGGL((k_coarse_parts<T, false>), grid, dim3(256), 0, st, g, U, x, xstride, parts, (T)m0,
                       half_dev, C);
  LQ_HIP(hipGetLastError());
}

template void launch_wilson<float>(const Geom &, const c64 *, const c64 *, c64 *, const c64 *, double,
                                   const Shifts &, int, int, hipStream_t, const c64 *);
template void launch_wilson<double>(const Geom &, const c128 *, const c128 *, c128 *, const c128 *, double,
                                    const Shifts &, int, int, hipStream_t, const c128 *);
template void launch_coarse_parts<float>(const Geom &, const c64 *, const c64 *, const int *, int, long long,
                                         c64 *, double, hipStream_t, const c64 *);
template void launch_coarse_parts<double>(const Geom &, const c128 *, const c128 *, const int *, int,
                                          long long, c128 *, double, hipStream_t, const c128 *);

}  // namespace lq
