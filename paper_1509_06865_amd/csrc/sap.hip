// Schwarz alternating procedure (SAP) smoother, one colour pass per launch.
//
// SAP is applied to D_sigma = gamma5 (Q - sigma) = D - sigma gamma5 with
// right-hand side gamma5 r, which with exact block solves gives the same
// iterates as SAP on Q - sigma (gamma5 is site-local), while its block
// systems are well suited to minimal-residual steps.  One workgroup owns one
// block (the lattice is stored blocked, so the block's sites are contiguous):
// it forms the block residual with the full stencil, runs the MR steps on the
// Dirichlet block operator with the iterate exchanged through LDS, and adds
// the correction to z.  Blocks of one colour never touch each other.
#include "lq_kernels.h"
#include "lq_dslash.h"

namespace lq {
namespace {

template <typename T> __device__ inline T wsumT(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Registers capped for four waves per SIMD (a few values spill; measured
// faster than three waves without spills: 0.179 against 0.186 ms per 16-field
// pass on 16^4).  With CLOV the site term carries the clover term.
template <typename T, bool CLOV>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1))) k_sap_colour(Geom g, const cplx<T> *__restrict__ U,
                                                    const cplx<T> *__restrict__ rin, cplx<T> *__restrict__ zio,
                                                    const int *__restrict__ blocks, T m0, Shifts sig, int n_mr,
                                                    int nrhs, const cplx<T> *__restrict__ C) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *lds = reinterpret_cast<cplx<T> *>(smem_raw);          // [12][bvol]
  __shared__ T red[4][3];                        // per-wave partial sums (<= 4 waves)
  // one workgroup per (block, rhs); the right-hand sides of one block are
  // consecutive tiles of one XCD, so its links are read from HBM once and
  // then come from that XCD's L2
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int B = blocks[tile / nrhs];
  const int k = tile - (tile / nrhs) * nrhs;
  const int t = threadIdx.x;
  const bool active = t < g.bvol;
  const int s = B * g.bvol + (active ? t : 0);
  const long long off = (long long)k * 12 * g.V;
  const cplx<T> *r = rin + off;
  cplx<T> *z = zio + off;
  const T sgm = (T)sig.s[k];
  const T diag = (T)4 + m0;
  // neighbour bookkeeping without runtime-indexed arrays (which would live
  // in scratch): per-thread bits for "the neighbour in direction mu lies in
  // the block" and uniform bits for "the block has a neighbour block in
  // direction mu without wrapping"
  int fmask = 0, bmask = 0, afw = 0;
  {
    int r = active ? t : 0, q = B;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int l = (mu < 3) ? r % g.b[mu] : r;
      r = (mu < 3) ? r / g.b[mu] : 0;
      const int a = (mu < 3) ? q % g.nb[mu] : q;
      q = (mu < 3) ? q / g.nb[mu] : 0;
      fmask |= (l + 1 < g.b[mu]) ? (1 << mu) : 0;
      bmask |= (l > 0) ? (1 << mu) : 0;
      afw |= (a + 1 < g.nb[mu]) ? (1 << mu) : 0;
    }
  }
  int abw = 0;
  {
    int q = B;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      const int a = (mu < 3) ? q % g.nb[mu] : q;
      q = (mu < 3) ? q / g.nb[mu] : 0;
      abw |= (a > 0) ? (1 << mu) : 0;
    }
  }

  // block residual rho = gamma5 r - D_sigma z (full stencil)
  cplx<T> rho[12], e[12], p[12], q[12];
  if (active) {
    cplx<T> acc[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      // uniform per-direction geometry (selects, no indexing)
      const int slm = mu == 0 ? g.sl[0] : mu == 1 ? g.sl[1] : mu == 2 ? g.sl[2] : g.sl[3];
      const int bm = mu == 0 ? g.b[0] : mu == 1 ? g.b[1] : mu == 2 ? g.b[2] : g.b[3];
      const int nbm = mu == 0 ? g.nb[0] : mu == 1 ? g.nb[1] : mu == 2 ? g.nb[2] : g.nb[3];
      const int sAm = mu == 0 ? g.sA[0] : mu == 1 ? g.sA[1] : mu == 2 ? g.sA[2] : g.sA[3];
      const long long jump = (long long)sAm * g.bvol;
      int sf, sb;
      T sgf = (T)1, sgb = (T)1;
      if ((fmask >> mu) & 1) {
        sf = s + slm;
      } else {
        sf = s - (bm - 1) * slm + (((afw >> mu) & 1) ? (int)jump : -(int)((nbm - 1) * jump));
        if (mu == 3 && !((afw >> 3) & 1)) sgf = (T)g.tbc;
      }
      if ((bmask >> mu) & 1) {
        sb = s - slm;
      } else {
        sb = s + (bm - 1) * slm + (((abw >> mu) & 1) ? -(int)jump : (int)((nbm - 1) * jump));
        if (mu == 3 && !((abw >> 3) & 1)) sgb = (T)g.tbc;
      }
#pragma unroll
      for (int i = 0; i < 12; ++i) q[i] = z[(long long)i * g.V + sf];
      hop(mu, true, q, U, g.V, s, sgf, acc);
#pragma unroll
      for (int i = 0; i < 12; ++i) q[i] = z[(long long)i * g.V + sb];
      hop(mu, false, q, U, g.V, sb, sgb, acc);
    }
    if constexpr (CLOV) {
#pragma unroll
      for (int i = 0; i < 12; ++i) q[i] = z[(long long)i * g.V + s];
      clover_add(C, g.V, s, q, (T)-2, acc);         // -1/2 acc then adds C z
    }
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const cplx<T> zi = z[(long long)i * g.V + s];
      const cplx<T> ri = r[(long long)i * g.V + s];
      const T g5 = (i < 6) ? (T)1 : (T)-1;
      // D_sigma z = (4+m0) z - acc/2 - sigma gamma5 z
      const cplx<T> dz = diag * zi - (T)0.5 * acc[i] - (sgm * g5) * zi;
      rho[i] = g5 * ri - dz;
      e[i] = mk<T>(0, 0);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 12; ++i) { rho[i] = mk<T>(0, 0); e[i] = mk<T>(0, 0); }
  }

  // MR steps on the block: rho lives in LDS so that block neighbours see it.
  // Two barriers per step: after the partial sums (all reads of the old rho
  // are done), and after the new rho is stored.  Sums are in T (FP32 for the
  // FP32 smoother).
  const int lane = t & 63, wave = t >> 6, nwv = blockDim.x >> 6;
  if (active)
#pragma unroll
    for (int i = 0; i < 12; ++i) lds[i * g.bvol + t] = rho[i];
  __syncthreads();
  for (int it = 0; it < n_mr; ++it) {
    T num_re = 0, num_im = 0, den = 0;
    if (active) {
      cplx<T> acc[12];
#pragma unroll
      for (int i = 0; i < 12; ++i) acc[i] = mk<T>(0, 0);
#pragma unroll 1
      for (int mu = 0; mu < 4; ++mu) {
        if ((fmask >> mu) & 1) {
          const int tn = t + (mu == 0 ? g.sl[0] : mu == 1 ? g.sl[1] : mu == 2 ? g.sl[2] : g.sl[3]);
#pragma unroll
          for (int i = 0; i < 12; ++i) q[i] = lds[i * g.bvol + tn];
          hop(mu, true, q, U, g.V, s, (T)1, acc);
        }
        if ((bmask >> mu) & 1) {
          const int slm = mu == 0 ? g.sl[0] : mu == 1 ? g.sl[1] : mu == 2 ? g.sl[2] : g.sl[3];
          const int tn = t - slm;
#pragma unroll
          for (int i = 0; i < 12; ++i) q[i] = lds[i * g.bvol + tn];
          hop(mu, false, q, U, g.V, s - slm, (T)1, acc);
        }
      }
      if constexpr (CLOV) clover_add(C, g.V, s, rho, (T)-2, acc);
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        const T g5 = (i < 6) ? (T)1 : (T)-1;
        p[i] = diag * rho[i] - (T)0.5 * acc[i] - (sgm * g5) * rho[i];
        // <p, rho> and <p, p>
        num_re += p[i].re * rho[i].re + p[i].im * rho[i].im;
        num_im += p[i].re * rho[i].im - p[i].im * rho[i].re;
        den += p[i].re * p[i].re + p[i].im * p[i].im;
      }
    }
    num_re = wsumT(num_re); num_im = wsumT(num_im); den = wsumT(den);
    if (lane == 0) { red[wave][0] = num_re; red[wave][1] = num_im; red[wave][2] = den; }
    __syncthreads();
    num_re = num_im = den = 0;
    for (int w = 0; w < nwv; ++w) { num_re += red[w][0]; num_im += red[w][1]; den += red[w][2]; }
    cplx<T> alpha = mk<T>(0, 0);
    if (den > 0) alpha = mk<T>(num_re / den, num_im / den);
    if (active)
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        e[i] = e[i] + alpha * rho[i];
        rho[i] = rho[i] - alpha * p[i];
        lds[i * g.bvol + t] = rho[i];
      }
    __syncthreads();
  }
  if (active)
#pragma unroll
    for (int i = 0; i < 12; ++i) z[(long long)i * g.V + s] = z[(long long)i * g.V + s] + e[i];
}

}  // namespace

template <typename T>
void launch_sap_colour(const Geom &g, const cplx<T> *U, const cplx<T> *r, cplx<T> *z, const int *blocks,
                       int nblocks, double m0, const Shifts &sig, int nrhs, int n_mr, hipStream_t st,
                       const cplx<T> *C) {
  if (nblocks <= 0 || nrhs <= 0) return;
  const int threads = ((g.bvol + 63) / 64) * 64;
  // algorithmic bytes: the colour's links (and clover blocks) once; per field
  // r, z of the colour's sites and of the other colour's (the blocks' halo), z out
  KTimerScope kt(KT_SAP, (double)nblocks * g.bvol * (36.0 + (C ? 42.0 : 0.0) + 48.0 * nrhs) * sizeof(cplx<T>));
  const size_t lds = (size_t)12 * g.bvol * sizeof(cplx<T>);
  if (C)
    LQ_LAUNCH(kt, (k_sap_colour<T, true>), dim3(nblocks * nrhs), dim3(threads), lds, st, g, U, r, z, blocks,
              (T)m0, sig, n_mr, nrhs, C);
  else
    LQ_LAUNCH(kt, (k_sap_colour<T, false>), dim3(nblocks * nrhs), dim3(threads), lds, st, g, U, r, z, blocks,
              (T)m0, sig, n_mr, nrhs, C);
  LQ_HIP(hipGetLastError());
}

template void launch_sap_colour<float>(const Geom &, const c64 *, const c64 *, c64 *, const int *, int, double,
                                       const Shifts &, int, int, hipStream_t, const c64 *);
template void launch_sap_colour<double>(const Geom &, const c128 *, const c128 *, c128 *, const int *, int,
                                        double, const Shifts &, int, int, hipStream_t, const c128 *);

}  // namespace lq
