// Clover term of the clover-improved Wilson-Dirac operator (sec. 2 names the
// operator; the standard Sheikholeslami-Wohlert form is taken):
//   C(x) = c_sw (i/4) sum_{mu != nu} sigma_munu (x) F_munu(x),
//   F_munu = (Q_munu - Q_munu^dag) / 8, Q_munu the four plaquettes of the
//   mu-nu plane that start and end at x (same orientation),
//   sigma_munu = (i/2) [gamma_mu, gamma_nu].
// In the chiral basis of the stencil, sigma_kl = -eps_klm s_m on both
// chiralities and sigma_kt = -s_k on the upper, +s_k on the lower one (s_m
// the Pauli matrices), so with eta = +1 (upper) or -1 (lower)
//   C_eta = c_sw (i/2) (s_1 (x) A_1 + s_2 (x) A_2 + s_3 (x) A_3),
//   A_1 = -F_yz - eta F_xt,  A_2 = F_xz - eta F_yt,  A_3 = -F_xy - eta F_zt.
// One thread per site builds both 6 x 6 blocks from the FP64 links (a setup
// step: the closed loops are formed directly, nothing is staged).
#include "lq_kernels.h"
#include "lq_dslash.h"

namespace lq {
namespace {

struct M3 { c128 e[9]; };

__device__ inline M3 mmul(const M3 &a, const M3 &b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = a.e[3 * i] * b.e[j] + a.e[3 * i + 1] * b.e[3 + j] + a.e[3 * i + 2] * b.e[6 + j];
  return r;
}

__device__ inline M3 mdag(const M3 &a) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.e[3 * i + j] = conj(a.e[3 * j + i]);
  return r;
}

__device__ inline M3 link(const c128 *__restrict__ U, long long V, int mu, int s) {
  M3 m;
#pragma unroll
  for (int k = 0; k < 9; ++k) m.e[k] = U[(long long)(mu * 9 + k) * V + s];
  return m;
}

__device__ inline int step(const Geom &g, int s, int mu, bool fwd) {
  const SiteCoord c = decode(g, s);
  float sg;
  bool in;
  return neighbour(g, s, c, mu, fwd, &sg, &in);     // gauge loops carry no boundary sign
}

// F_munu(x) = (Q - Q^dag) / 8 with Q the sum of the four leaves at x
__device__ inline M3 field_strength(const Geom &g, const c128 *__restrict__ U, int s, int mu, int nu) {
  const long long V = g.V;
  const int xm = step(g, s, mu, true), xn = step(g, s, nu, true);
  const int xmm = step(g, s, mu, false), xnm = step(g, s, nu, false);
  const int x_mm_n = step(g, xmm, nu, true), x_mm_nm = step(g, xmm, nu, false), x_nm_m = step(g, xnm, mu, true);
  const M3 Um = link(U, V, mu, s), Un = link(U, V, nu, s);
  M3 Q = mmul(mmul(Um, link(U, V, nu, xm)), mdag(mmul(Un, link(U, V, mu, xn))));
  const M3 Umm = link(U, V, mu, xmm), Unn = link(U, V, nu, xnm);
  const M3 p2 = mmul(mmul(Un, mdag(link(U, V, mu, x_mm_n))), mmul(mdag(link(U, V, nu, xmm)), Umm));
  const M3 p3 = mmul(mmul(mdag(Umm), mdag(link(U, V, nu, x_mm_nm))), mmul(link(U, V, mu, x_mm_nm), Unn));
  const M3 p4 = mmul(mmul(mdag(Unn), link(U, V, mu, xnm)), mmul(link(U, V, nu, x_nm_m), mdag(Um)));
  M3 F;
#pragma unroll
  for (int k = 0; k < 9; ++k) Q.e[k] = Q.e[k] + p2.e[k] + p3.e[k] + p4.e[k];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) F.e[3 * i + j] = 0.125 * (Q.e[3 * i + j] - conj(Q.e[3 * j + i]));
  return F;
}

__global__ void __launch_bounds__(128) k_clover_build(Geom g, const c128 *__restrict__ U, double csw,
                                                      c128 *__restrict__ C) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.V) return;
  const long long V = g.V;
  // planes xy, xz, xt, yz, yt, zt
  M3 F[6];
  F[0] = field_strength(g, U, s, 0, 1);
  F[1] = field_strength(g, U, s, 0, 2);
  F[2] = field_strength(g, U, s, 0, 3);
  F[3] = field_strength(g, U, s, 1, 2);
  F[4] = field_strength(g, U, s, 1, 3);
  F[5] = field_strength(g, U, s, 2, 3);
  const c128 pre = mk(0.0, 0.5 * csw);                 // c_sw i / 2
  for (int b = 0; b < 2; ++b) {
    const double eta = b == 0 ? 1.0 : -1.0;
    M3 A1, A2, A3;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      A1.e[k] = -F[3].e[k] - eta * F[2].e[k];
      A2.e[k] = F[1].e[k] - eta * F[4].e[k];
      A3.e[k] = -F[0].e[k] - eta * F[5].e[k];
    }
    // 2 x 2 spin blocks: (0,0) A3, (0,1) A1 - i A2, (1,0) A1 + i A2, (1,1) -A3
    auto entry = [&](int k, int l) -> c128 {
      const int sk = k / 3, a = k % 3, sl = l / 3, c = l % 3;
      const c128 a1 = A1.e[3 * a + c], a2 = A2.e[3 * a + c], a3 = A3.e[3 * a + c];
      c128 v;
      if (sk == 0 && sl == 0) v = a3;
      else if (sk == 0) v = a1 - times_i(a2);
      else if (sl == 0) v = a1 + times_i(a2);
      else v = -a3;
      return pre * v;
    };
    c128 *Cb = C + (long long)(21 * b) * V + s;
    for (int k = 0; k < 6; ++k) Cb[(long long)k * V] = mk(entry(k, k).re, 0.0);
    int q = 6;
    for (int k = 0; k < 6; ++k)
      for (int l = k + 1; l < 6; ++l) Cb[(long long)(q++) * V] = entry(k, l);
  }
  for (int r = 42; r < kCloverRows; ++r) C[(long long)r * V + s] = mk(0.0, 0.0);
}

}  // namespace

void launch_clover_build(const Geom &g, const c128 *U, double csw, c128 *C, hipStream_t st) {
  hipLaunchKernelGGL(k_clover_build, dim3(blocks_for(g.V, 128)), dim3(128), 0, st, g, U, csw, C);
  LQ_HIP(hipGetLastError());
}

}  // namespace lq
