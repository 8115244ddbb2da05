// Device helpers for the Wilson hop terms, shared by the stencil, the SAP
// smoother and the coarse-operator build.
//
// In the chiral basis gamma_mu = [[0, A_mu], [A_mu^dag, 0]] with A_k = i sigma_k
// (k = x, y, z) and A_t = 1, the projected spinor (1 + e gamma_mu) psi
// (e = -1 for the forward hop, +1 for the backward hop) is fixed by its upper
// half h = psi_u + e A_mu psi_l; its lower half is e A_mu^dag h.  Only h (two
// spins) is multiplied by the link, which halves the SU(3) work.
#pragma once
#include "lq_common.h"

namespace lq {

template <typename T> struct Half2 { cplx<T> v[2][3]; };

template <typename T>
__device__ inline void load_link(const cplx<T> *__restrict__ U, long long V, int mu, int s, cplx<T> m[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = U[(long long)(mu * 9 + k) * V + s];
}

template <typename T>
__device__ inline void load_spinor(const cplx<T> *__restrict__ x, long long V, int s, cplx<T> p[12]) {
#pragma unroll
  for (int k = 0; k < 12; ++k) p[k] = x[(long long)k * V + s];
}

// Upper half of (1 + e gamma_mu) psi.
template <typename T>
__device__ inline void project(int mu, T e, const cplx<T> p[12], Half2<T> &h) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<T> p0 = p[c], p1 = p[3 + c], p2 = p[6 + c], p3 = p[9 + c];
    switch (mu) {
      case 0: h.v[0][c] = p0 + e * times_i(p3); h.v[1][c] = p1 + e * times_i(p2); break;
      case 1: h.v[0][c] = p0 + e * p3;          h.v[1][c] = p1 - e * p2;          break;
      case 2: h.v[0][c] = p0 + e * times_i(p2); h.v[1][c] = p1 - e * times_i(p3); break;
      default: h.v[0][c] = p0 + e * p2;         h.v[1][c] = p1 + e * p3;          break;
    }
  }
}

// acc += sign * (upper u, lower e A_mu^dag u)
template <typename T>
__device__ inline void reconstruct(int mu, T e, const Half2<T> &u, T sign, cplx<T> acc[12]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cplx<T> u0 = sign * u.v[0][c], u1 = sign * u.v[1][c];
    acc[c] = acc[c] + u0;
    acc[3 + c] = acc[3 + c] + u1;
    switch (mu) {
      case 0: acc[6 + c] = acc[6 + c] - e * times_i(u1); acc[9 + c] = acc[9 + c] - e * times_i(u0); break;
      case 1: acc[6 + c] = acc[6 + c] - e * u1;          acc[9 + c] = acc[9 + c] + e * u0;          break;
      case 2: acc[6 + c] = acc[6 + c] - e * times_i(u0); acc[9 + c] = acc[9 + c] + e * times_i(u1); break;
      default: acc[6 + c] = acc[6 + c] + e * u0;         acc[9 + c] = acc[9 + c] + e * u1;          break;
    }
  }
}

// u = M h (dag = false) or M^dag h (dag = true), M row-major 3x3, per spin.
template <typename T>
__device__ inline void link_mul(const cplx<T> m[9], const Half2<T> &h, Half2<T> &u, bool dag) {
#pragma unroll
  for (int sp = 0; sp < 2; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cplx<T> acc;
      if (!dag) acc = m[3 * a] * h.v[sp][0] + m[3 * a + 1] * h.v[sp][1] + m[3 * a + 2] * h.v[sp][2];
      else acc = cmul_conj(m[a], h.v[sp][0]) + cmul_conj(m[3 + a], h.v[sp][1]) + cmul_conj(m[6 + a], h.v[sp][2]);
      u.v[sp][a] = acc;
    }
}

// acc += sign * (1 - gamma_mu) m p        (fwd = true)
// acc += sign * (1 + gamma_mu) m^dag p    (fwd = false), m a loaded link
template <typename T>
__device__ inline void hop_link(int mu, bool fwd, const cplx<T> p[12], const cplx<T> m[9], T sign, cplx<T> acc[12]) {
  const T e = fwd ? (T)-1 : (T)1;
  Half2<T> h, u;
  project(mu, e, p, h);
  link_mul(m, h, u, !fwd);
  reconstruct(mu, e, u, sign, acc);
}

// acc += sign * (1 - gamma_mu) U_mu(link_site) p        (fwd = true)
// acc += sign * (1 + gamma_mu) U_mu(link_site)^dag p    (fwd = false)
template <typename T>
__device__ inline void hop(int mu, bool fwd, const cplx<T> p[12], const cplx<T> *__restrict__ U, long long V,
                           int link_site, T sign, cplx<T> acc[12]) {
  cplx<T> m[9];
  load_link(U, V, mu, link_site, m);
  hop_link(mu, fwd, p, m, sign, acc);
}

// Clover term (site-local, commutes with gamma5): per site two Hermitian 6 x 6
// blocks, one per chirality (components 6b .. 6b + 5 = spins 2b, 2b + 1 times
// colour).  Stored [48][V] (42 used): block b at rows 21 b .. 21 b + 20, the
// six diagonal entries (real, held in .re) first, then the upper triangle
// (k, l), k < l, row by row (kCloverRows in lq_common.h).

// acc += scale * C(s) p
template <typename T>
__device__ inline void clover_add(const cplx<T> *__restrict__ C, long long V, int s, const cplx<T> p[12], T scale,
                                  cplx<T> acc[12]) {
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const cplx<T> *Cb = C + (long long)(21 * b) * V + s;
    cplx<T> y[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) y[k] = Cb[(long long)k * V].re * p[6 * b + k];
    int q = 6;
#pragma unroll
    for (int k = 0; k < 6; ++k)
#pragma unroll
      for (int l = k + 1; l < 6; ++l) {
        const cplx<T> m = Cb[(long long)q * V];
        y[k] = y[k] + m * p[6 * b + l];
        y[l] = y[l] + cmul_conj(m, p[6 * b + k]);
        ++q;
      }
#pragma unroll
    for (int k = 0; k < 6; ++k) acc[6 * b + k] = acc[6 * b + k] + scale * y[k];
  }
}

}  // namespace lq
