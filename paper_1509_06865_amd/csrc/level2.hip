// The third multigrid level: aggregation of the coarse lattice.  Level-1
// vectors are [n][nA1][2 Nv1] (coarse sites in canonical order, x fastest;
// entry h*Nv1 + c of a site is component c of gamma5^c half h).  Level-2
// aggregates are blocks of extent b2 of the coarse lattice.  P2 is stored as
// Nv2 level-1 vectors; its restriction to (level-2 aggregate A2, half h) gives
// the orthonormal columns (A2, h, k), so gamma5^c P2 = P2 gamma5^c2 and
// P2^dag P2 = 1 as on the first level (sec. 2's construction applied once
// more).  Q_c2 = P2^dag Q_c P2 is stored like Q_c, so the coarse-apply
// kernels serve both levels.
#include "lq_kernels.h"

namespace lq {
namespace {

__device__ inline double wsum2(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// level-1 site of local index l in level-2 aggregate A2
__device__ inline int l2_site(const Level2Geom &g, int A2, int l) {
  int a1[4];
  int q = A2, r = l;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int a2 = (mu < 3) ? q % g.nb2[mu] : q;
    q = (mu < 3) ? q / g.nb2[mu] : 0;
    const int lc = (mu < 3) ? r % g.b2[mu] : r;
    r = (mu < 3) ? r / g.b2[mu] : 0;
    a1[mu] = a2 * g.b2[mu] + lc;
  }
  return a1[0] + g.nb1[0] * (a1[1] + g.nb1[1] * (a1[2] + g.nb1[2] * a1[3]));
}

// level-2 aggregate of level-1 site A1
__device__ inline int l2_agg(const Level2Geom &g, int A1) {
  int q = A1, A2 = 0, stride = 1;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const int a1 = (mu < 3) ? q % g.nb1[mu] : q;
    q = (mu < 3) ? q / g.nb1[mu] : 0;
    A2 += (a1 / g.b2[mu]) * stride;
    stride *= g.nb2[mu];
  }
  return A2;
}

// c2[j][A2][h Nv2 + k] = sum over the aggregate's sites and half-h entries of
// conj(P2_k) v_j.  One workgroup per (A2, h); thread (k, j) accumulates one
// output while the rows pass through LDS in chunks of 32.
constexpr int kR2Chunk = 32;
template <typename T>
__global__ void __launch_bounds__(512) k_restrict2(Level2Geom g, const cplx<T> *__restrict__ P2,
                                                   const cplx<T> *__restrict__ v, int nrhs,
                                                   cplx<T> *__restrict__ c2) {
  __shared__ cplx<T> ps[kR2Chunk][32];
  __shared__ cplx<T> vs[kR2Chunk][kMaxRhs];
  const int A2 = blockIdx.x, h = blockIdx.y;
  const int t = threadIdx.x, nthr = blockDim.x;
  const int Nv1 = g.Nv1, Nv2 = g.Nv2, n21 = 2 * Nv1;
  const int k = t % Nv2, j = t / Nv2;
  const int m = g.bvol2 * Nv1;
  cplx<T> acc = mk<T>(0, 0);
  for (int e0 = 0; e0 < m; e0 += kR2Chunk) {
    __syncthreads();
    for (int q = t; q < kR2Chunk * (Nv2 + nrhs); q += nthr) {
      const int e = q % kR2Chunk, col = q / kR2Chunk;
      const int ee = e0 + e;
      cplx<T> val = mk<T>(0, 0);
      if (ee < m) {
        const int l = ee / Nv1, cc = ee - l * Nv1;
        const long long site = l2_site(g, A2, l);
        if (col < Nv2) val = P2[((long long)col * g.nA1 + site) * n21 + h * Nv1 + cc];
        else val = v[((long long)(col - Nv2) * g.nA1 + site) * n21 + h * Nv1 + cc];
      }
      if (col < Nv2) ps[e][col] = val;
      else vs[e][col - Nv2] = val;
    }
    __syncthreads();
    if (j < nrhs)
#pragma unroll 8
      for (int e = 0; e < kR2Chunk; ++e) acc = acc + cmul_conj(ps[e][k], vs[e][j]);
  }
  if (j < nrhs) c2[((long long)j * g.nA2 + A2) * (2 * Nv2) + h * Nv2 + k] = acc;
}

// v_j (+)= P2 c2_j.  One workgroup per A2: the aggregate's coarse entries of
// every rhs in LDS, one thread per (site, entry) of the aggregate.
template <typename T>
__global__ void __launch_bounds__(256) k_prolong2(Level2Geom g, const cplx<T> *__restrict__ P2,
                                                  const cplx<T> *__restrict__ c2, cplx<T> *__restrict__ v, int nrhs,
                                                  bool accumulate) {
  __shared__ cplx<T> cs[kMaxRhs][64];
  const int A2 = blockIdx.x, t = threadIdx.x;
  const int Nv1 = g.Nv1, Nv2 = g.Nv2, n21 = 2 * Nv1, n22 = 2 * Nv2;
  for (int q = t; q < nrhs * n22; q += blockDim.x) {
    const int j = q / n22, e = q - j * n22;
    cs[j][e] = c2[((long long)j * g.nA2 + A2) * n22 + e];
  }
  __syncthreads();
  for (int q = t; q < g.bvol2 * n21; q += blockDim.x) {
    const int l = q / n21, i = q - l * n21;
    const int h = i / Nv1;
    const long long site = l2_site(g, A2, l);
    cplx<T> out[kMaxRhs];
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) out[j] = mk<T>(0, 0);
    for (int k = 0; k < Nv2; ++k) {
      const cplx<T> p = P2[((long long)k * g.nA1 + site) * n21 + i];
#pragma unroll
      for (int j = 0; j < kMaxRhs; ++j)
        if (j < nrhs) out[j] = out[j] + p * cs[j][h * Nv2 + k];
    }
#pragma unroll
    for (int j = 0; j < kMaxRhs; ++j) {
      if (j >= nrhs) break;
      const long long e = ((long long)j * g.nA1 + site) * n21 + i;
      v[e] = accumulate ? v[e] + out[j] : out[j];
    }
  }
}

// P2 from level-1 test vectors W (FP64): per (A2, h) Cholesky-QR applied
// twice to the (bvol2 Nv1) x Nv2 local matrix, as for the first level's P.
// Columns that are dependent there (a pivot below 1e-13 of its diagonal)
// leave that block of P2 unwritten and raise *status.
constexpr int kMaxNv2 = 32;
__global__ void __launch_bounds__(256) k_build_P2(Level2Geom g, const c128 *__restrict__ W, c128 *__restrict__ P,
                                                  int *status) {
  __shared__ double part[4][2];
  __shared__ c128 L[kMaxNv2][kMaxNv2];
  __shared__ int bad;
  const int A2 = blockIdx.x, h = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const int Nv1 = g.Nv1, Nv = g.Nv2, n21 = 2 * Nv1;
  const int m = g.bvol2 * Nv1;
  auto addr = [&](int col, int e) -> long long {
    const int l = e / Nv1, cc = e - l * Nv1;
    return ((long long)col * g.nA1 + l2_site(g, A2, l)) * n21 + h * Nv1 + cc;
  };
  if (t == 0) bad = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const c128 *src = (pass == 0) ? W : P;
    // Gram entries G[j][i] = <w_j, w_i> for i >= j, one reduction each
    for (int i = 0; i < Nv; ++i)
      for (int jj = i; jj < Nv; ++jj) {
        double re = 0, im = 0;
        for (int e = t; e < m; e += blockDim.x) {
          const c128 a = src[addr(i, e)], b = src[addr(jj, e)];
          re += a.re * b.re + a.im * b.im;
          im += a.re * b.im - a.im * b.re;
        }
        re = wsum2(re);
        im = wsum2(im);
        __syncthreads();
        if (lane == 0) { part[wave][0] = re; part[wave][1] = im; }
        __syncthreads();
        if (t == 0) {
          double sr = 0, si = 0;
          for (int w = 0; w < nw; ++w) { sr += part[w][0]; si += part[w][1]; }
          L[jj][i] = c128{sr, -si};                 // lower triangle: G[j][i] = conj(<w_i, w_j>)
        }
      }
    __syncthreads();
    if (t == 0) {
      for (int jj = 0; jj < Nv; ++jj) {
        const double gjj = L[jj][jj].re;
        double d = gjj;
        for (int k = 0; k < jj; ++k) d -= norm2(L[jj][k]);
        if (!(d > 1e-13 * gjj) || !(gjj > 0)) { bad = 1; break; }
        const double ljj = sqrt(d);
        L[jj][jj] = c128{ljj, 0};
        for (int i = jj + 1; i < Nv; ++i) {
          c128 v = L[i][jj];
          for (int k = 0; k < jj; ++k) v = v - cmul_conj(L[jj][k], L[i][k]);
          L[i][jj] = (1.0 / ljj) * v;
        }
      }
    }
    __syncthreads();
    if (bad) break;
    // rows: p = w L^-dag
    for (int e = t; e < m; e += blockDim.x) {
      c128 pr[kMaxNv2];
      for (int jj = 0; jj < Nv; ++jj) {
        c128 v = src[addr(jj, e)];
        for (int i = 0; i < jj; ++i) v = v - pr[i] * conj(L[jj][i]);
        pr[jj] = (1.0 / L[jj][jj].re) * v;
      }
      for (int jj = 0; jj < Nv; ++jj) P[addr(jj, e)] = pr[jj];
    }
    __syncthreads();
  }
  if (t == 0 && bad) atomicOr(status, 1);
}

__device__ inline int cnbr1(const int nb[4], int A, int mu, int step) {
  int a[4], r = A;
  for (int m = 0; m < 3; ++m) { a[m] = r % nb[m]; r /= nb[m]; }
  a[3] = r;
  a[mu] = (a[mu] + step + nb[mu]) % nb[mu];
  return a[0] + nb[0] * (a[1] + nb[1] * (a[2] + nb[2] * a[3]));
}

// Split couplings of Q_c for the level-2 operator.  Input: nc columns x_q
// (level-1 vectors; x_q = P2_l with half half[q] only).  Output
// parts[q][5][nA1][2 Nv1]: part 0 = the couplings whose source and target lie
// in one level-2 aggregate, part 1 + mu = the forward couplings in mu that
// leave the target's aggregate (source in the next aggregate).  One thread per
// (q, A1, row).
template <typename T>
__global__ void k_coarse_parts2(Level2Geom g, const cplx<T> *__restrict__ Qc, const cplx<T> *__restrict__ x,
                                const int *__restrict__ half, int nc, long long xstride,
                                cplx<T> *__restrict__ parts) {
  const int Nv1 = g.Nv1, n2 = 2 * Nv1;
  const long long tot = (long long)nc * g.nA1 * n2;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= tot) return;
  const int i = (int)(e % n2);
  const int A1 = (int)((e / n2) % g.nA1);
  const int q = (int)(e / ((long long)n2 * g.nA1));
  const cplx<T> *xq = x + q * xstride;
  const int h = half[q];
  const long long bs = (long long)n2 * n2;
  // local coordinates of A1 inside its level-2 aggregate
  int lc[4];
  {
    int r = A1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int a1 = (mu < 3) ? r % g.nb1[mu] : r;
      r = (mu < 3) ? r / g.nb1[mu] : 0;
      lc[mu] = a1 % g.b2[mu];
    }
  }
  cplx<T> self = mk<T>(0, 0), fwd[4];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) fwd[mu] = mk<T>(0, 0);
  // only the source entries of half h are non-zero
  const int j0 = h * Nv1, j1 = j0 + Nv1;
  {
    const cplx<T> *M = Qc + ((long long)A1 * 5) * bs + (long long)i * n2;
    const cplx<T> *xs = xq + (long long)A1 * n2;
    for (int j = j0; j < j1; ++j) self = self + M[j] * xs[j];
  }
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    // forward: Qc[A1][1 + mu] x(A1 + mu)
    const int B = cnbr1(g.nb1, A1, mu, 1);
    const cplx<T> *M = Qc + ((long long)A1 * 5 + 1 + mu) * bs + (long long)i * n2;
    const cplx<T> *xs = xq + (long long)B * n2;
    cplx<T> s = mk<T>(0, 0);
    for (int j = j0; j < j1; ++j) s = s + M[j] * xs[j];
    if (lc[mu] + 1 < g.b2[mu]) self = self + s;
    else fwd[mu] = s;
    // backward: Qc[A1 - mu][1 + mu]^dag x(A1 - mu); it stays inside the aggregate
    // unless A1 is on its backward face (then it belongs to the backward block,
    // which is not stored)
    if (lc[mu] > 0) {
      const int Bb = cnbr1(g.nb1, A1, mu, -1);
      const cplx<T> *Mb = Qc + ((long long)Bb * 5 + 1 + mu) * bs + i;
      const cplx<T> *xb = xq + (long long)Bb * n2;
      cplx<T> sb = mk<T>(0, 0);
      for (int j = j0; j < j1; ++j) sb = sb + cmul_conj(Mb[(long long)j * n2], xb[j]);
      self = self + sb;
    }
  }
  const long long ps = (long long)g.nA1 * n2;
  cplx<T> *pq = parts + (long long)q * 5 * ps + (long long)A1 * n2 + i;
  pq[0] = self;
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) pq[(1 + mu) * ps] = fwd[mu];
}

}  // namespace

template <typename T>
void launch_restrict2(const Level2Geom &g, const cplx<T> *P2, const cplx<T> *v, int nrhs, cplx<T> *c2,
                      hipStream_t st) {
  if (nrhs < 1 || nrhs > kMaxRhs || g.Nv2 > 32)
    throw HipError(hipErrorInvalidValue, "launch_restrict2: 1 <= nrhs <= 16, Nv2 <= 32", __FILE__, __LINE__);
  const int threads = ((g.Nv2 * nrhs + 63) / 64) * 64;
  hipLaunchKernelGGL((k_restrict2<T>), dim3(g.nA2, 2), dim3(threads), 0, st, g, P2, v, nrhs, c2);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_prolong2(const Level2Geom &g, const cplx<T> *P2, const cplx<T> *c2, cplx<T> *v, int nrhs,
                     bool accumulate, hipStream_t st) {
  if (nrhs < 1 || nrhs > kMaxRhs || 2 * g.Nv2 > 64)
    throw HipError(hipErrorInvalidValue, "launch_prolong2: 1 <= nrhs <= 16, Nv2 <= 32", __FILE__, __LINE__);
  hipLaunchKernelGGL((k_prolong2<T>), dim3(g.nA2), dim3(256), 0, st, g, P2, c2, v, nrhs, accumulate);
  LQ_HIP(hipGetLastError());
}

void launch_build_P2(const Level2Geom &g, const c128 *W, c128 *P2, int *status, hipStream_t st) {
  if (g.Nv2 > kMaxNv2) throw HipError(hipErrorInvalidValue, "launch_build_P2: Nv2 <= 32", __FILE__, __LINE__);
  hipLaunchKernelGGL(k_build_P2, dim3(g.nA2, 2), dim3(256), 0, st, g, W, P2, status);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_coarse_parts2(const Level2Geom &g, const cplx<T> *Qc, const cplx<T> *x, const int *half_dev, int nc,
                          long long xstride, cplx<T> *parts, hipStream_t st) {
  const long long tot = (long long)nc * g.nA1 * 2 * g.Nv1;
  hipLaunchKernelGGL((k_coarse_parts2<T>), dim3(blocks_for(tot, 256)), dim3(256), 0, st, g, Qc, x, half_dev, nc,
                     xstride, parts);
  LQ_HIP(hipGetLastError());
}

#define LQ_INST(T)                                                                                             \
  template void launch_restrict2<T>(const Level2Geom &, const cplx<T> *, const cplx<T> *, int, cplx<T> *,     \
                                    hipStream_t);                                                             \
  template void launch_prolong2<T>(const Level2Geom &, const cplx<T> *, const cplx<T> *, cplx<T> *, int, bool, \
                                   hipStream_t);                                                              \
  template void launch_coarse_parts2<T>(const Level2Geom &, const cplx<T> *, const cplx<T> *, const int *, int, \
                                        long long, cplx<T> *, hipStream_t);
LQ_INST(float)
LQ_INST(double)
#undef LQ_INST

}  // namespace lq
