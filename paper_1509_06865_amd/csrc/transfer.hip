// Grid transfers of the aggregation multigrid (sec. 2): the gamma5-split
// interpolation P = diag(P1, P2), restriction R = P^dag, prolongation, the
// local orthonormalisation that builds P from test vectors, and the scatter of
// restricted split hops into the Galerkin operator Q_c = P^dag Q P.
//
// The fine lattice is stored blocked by aggregate, so one workgroup owns the
// contiguous sites of one aggregate; P is stored as Nv fields in the same
// layout, its restriction to (aggregate, gamma5 half) being one column.
#include "lq_kernels.h"

namespace lq {
namespace {

// Wave sum of N values per lane (N a power of two, at most 64) by a transposed
// butterfly: at offset o each lane keeps half of its values, hands the other
// half to lane ^ o and adds what it receives, so N values cost N - 1 shuffles
// before the last log2(64 / N) plain steps.  Afterwards every lane holds the
// complete sum of value (lane / (64 / N)).
template <typename T, int N, int C, int O>
__device__ inline void transpose_step(T (&v)[N], int lane) {
  if constexpr (C > 1) {
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int j = 0; j < C / 2; ++j) {
      const T give = up ? v[j] : v[j + C / 2];
      const T keep = up ? v[j + C / 2] : v[j];
      v[j] = keep + __shfl_xor(give, O, 64);
    }
    transpose_step<T, N, C / 2, O / 2>(v, lane);
  }
}

template <typename T, int N>
__device__ inline T transpose_reduce(T (&v)[N], int lane) {
  transpose_step<T, N, N, 32>(v, lane);
  T x = v[0];
#pragma unroll
  for (int o = 32 / N; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// c[j][A][h*Nv + k] = sum over the aggregate's sites of conj(P_k) . f_j on half h.
// One workgroup per (aggregate, group of R fields): each P_k value is loaded
// once for the R fields held in registers.  Per k a lane forms 4R partial sums
// (field, half, re/im); a transposed butterfly reduces them over the wave and
// the waves' results meet in LDS.
template <typename T, int R>
__global__ void __launch_bounds__(256) k_restrict(Geom g, const cplx<T> *__restrict__ P, int Nv,
                                                  const cplx<T> *__restrict__ f, long long fstride, int nf,
                                                  cplx<T> *__restrict__ c) {
  constexpr int NV = 4 * R;
  __shared__ T part[4][32][NV];          // [wave][k][field * 4 + half * 2 + re/im]
  const int A = blockIdx.x, j0 = blockIdx.y * R;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const bool active = t < g.bvol;
  // idle lanes read a valid site and hold zero fields, so their products vanish
  const int s = A * g.bvol + (active ? t : 0);
  cplx<T> fv[R][12];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < 12; ++i)
      fv[r][i] = (active && j0 + r < nf) ? f[(j0 + r) * fstride + (long long)i * g.V + s] : mk<T>(0, 0);
  for (int k = 0; k < Nv; ++k) {
    cplx<T> pv[12];
    const cplx<T> *Pk = P + (long long)k * 12 * g.V;
#pragma unroll
    for (int i = 0; i < 12; ++i) pv[i] = Pk[(long long)i * g.V + s];
    T v[NV];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      T a0r = 0, a0i = 0, a1r = 0, a1i = 0;
#pragma unroll
      for (int i = 0; i < 12; ++i) {
        const T re = pv[i].re * fv[r][i].re + pv[i].im * fv[r][i].im;
        const T im = pv[i].re * fv[r][i].im - pv[i].im * fv[r][i].re;
        if (i < 6) { a0r += re; a0i += im; } else { a1r += re; a1i += im; }
      }
      v[4 * r + 0] = a0r; v[4 * r + 1] = a0i; v[4 * r + 2] = a1r; v[4 * r + 3] = a1i;
    }
    const T sum = transpose_reduce<T, NV>(v, lane);
    if ((lane & (64 / NV - 1)) == 0) part[wave][k][lane / (64 / NV)] = sum;
  }
  __syncthreads();
  const int n2 = 2 * Nv;
  for (int q = t; q < R * n2; q += blockDim.x) {
    const int r = q / n2, e = q - r * n2;
    if (j0 + r >= nf) continue;
    const int h = e / Nv, k = e - h * Nv;
    T re = 0, im = 0;
    for (int w = 0; w < nw; ++w) { re += part[w][k][4 * r + 2 * h]; im += part[w][k][4 * r + 2 * h + 1]; }
    c[((long long)(j0 + r) * g.nblk + A) * n2 + e] = mk<T>(re, im);
  }
}

// f_j(x) (+)= sum_k P_k(x) c_j[A][h(x) Nv + k], R fields per workgroup
template <typename T, int R>
__global__ void __launch_bounds__(256) k_prolong(Geom g, const cplx<T> *__restrict__ P, int Nv,
                                                 const cplx<T> *__restrict__ c, cplx<T> *__restrict__ f,
                                                 long long fstride, int nf, bool acc) {
  __shared__ cplx<T> cs[R][64];
  const int A = blockIdx.x, j0 = blockIdx.y * R;
  const int t = threadIdx.x;
  const int n2 = 2 * Nv;
  for (int q = t; q < R * n2; q += blockDim.x) {
    const int r = q / n2, e = q - r * n2;
    cs[r][e] = (j0 + r < nf) ? c[((long long)(j0 + r) * g.nblk + A) * n2 + e] : mk<T>(0, 0);
  }
  __syncthreads();
  if (t >= g.bvol) return;
  const int s = A * g.bvol + t;
  cplx<T> out[R][12];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int i = 0; i < 12; ++i) out[r][i] = mk<T>(0, 0);
  for (int k = 0; k < Nv; ++k) {
    const cplx<T> *Pk = P + (long long)k * 12 * g.V;
    cplx<T> pv[12];
#pragma unroll
    for (int i = 0; i < 12; ++i) pv[i] = Pk[(long long)i * g.V + s];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const cplx<T> c0 = cs[r][k], c1 = cs[r][Nv + k];
#pragma unroll
      for (int i = 0; i < 12; ++i) out[r][i] = out[r][i] + pv[i] * (i < 6 ? c0 : c1);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (j0 + r >= nf) break;
    cplx<T> *fj = f + (j0 + r) * fstride;
#pragma unroll
    for (int i = 0; i < 12; ++i) {
      const long long e = (long long)i * g.V + s;
      fj[e] = acc ? fj[e] + out[r][i] : out[r][i];
    }
  }
}

// fields per workgroup of the transfer kernels: 4 in FP32, 2 in FP64 (registers)
template <typename T> constexpr int transfer_group() { return sizeof(T) == 4 ? 4 : 2; }

// Cholesky-QR, applied twice, of the (6*bvol) x Nv local matrix of aggregate
// A and gamma5 half h.  Gram G = W^dag W, G = L L^dag, P = W L^-dag; the QR
// factor with positive diagonal is unique, so this is the same orthonormal
// basis that Gram-Schmidt in vector order produces.  If the columns are
// linearly dependent on the aggregate half (a pivot below 1e-13 of its
// diagonal), the workgroup writes nothing, so that block of P keeps its
// previous columns, and raises *status.
constexpr int kMaxNv = 32;
constexpr int kGramBatch = 8;                    // Gram entries whose wave sums run interleaved
__global__ void __launch_bounds__(256) k_build_P(Geom g, const c128 *const *__restrict__ cols, int Nv,
                                                 c128 *__restrict__ P, int *status) {
  __shared__ double part[4][kMaxNv * (kMaxNv + 1) / 2 * 2];   // wave partial sums of the Gram entries
  __shared__ c128 L[kMaxNv][kMaxNv];
  __shared__ int bad;
  const int A = blockIdx.x, h = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, nw = blockDim.x >> 6;
  const bool active = t < g.bvol;
  const int s = A * g.bvol + (active ? t : 0);
  const int npair = Nv * (Nv + 1) / 2;
  if (t == 0) bad = 0;
  for (int pass = 0; pass < 2; ++pass) {
    // field k of this pass: test vector k (its own address), then column k of P
    auto field = [&](int k) -> const c128 * { return (pass == 0) ? cols[k] : P + (long long)k * 12 * g.V; };
    // Gram partials, pairs (i <= j) in row-major order; the wave sums of
    // kGramBatch entries at a time run interleaved
    int pbase = 0;
#pragma unroll 1
    for (int i = 0; i < Nv; ++i) {
      c128 wi[6];
      const c128 *fi = field(i);
#pragma unroll
      for (int r = 0; r < 6; ++r)
        wi[r] = active ? fi[(long long)(6 * h + r) * g.V + s] : c128{0, 0};
#pragma unroll 1
      for (int j0 = i; j0 < Nv; j0 += kGramBatch) {
        double re[kGramBatch], im[kGramBatch];
#pragma unroll
        for (int b = 0; b < kGramBatch; ++b) {
          re[b] = 0;
          im[b] = 0;
          if (active && j0 + b < Nv) {
            const c128 *fj = field(j0 + b);
#pragma unroll
            for (int r = 0; r < 6; ++r) {
              const c128 wj = fj[(long long)(6 * h + r) * g.V + s];
              re[b] += wi[r].re * wj.re + wi[r].im * wj.im;
              im[b] += wi[r].re * wj.im - wi[r].im * wj.re;
            }
          }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
          for (int b = 0; b < kGramBatch; ++b) {
            re[b] += __shfl_xor(re[b], off, 64);
            im[b] += __shfl_xor(im[b], off, 64);
          }
        if (lane == 0) {
#pragma unroll
          for (int b = 0; b < kGramBatch; ++b)
            if (j0 + b < Nv) {
              const int q = pbase + j0 + b - i;
              part[wave][2 * q] = re[b];
              part[wave][2 * q + 1] = im[b];
            }
        }
      }
      pbase += Nv - i;
    }
    __syncthreads();
    // Gram matrix into L (upper part, then Cholesky in place by thread 0)
    for (int q = t; q < npair; q += blockDim.x) {
      int i = 0, rem = q;
      while (rem >= Nv - i) { rem -= Nv - i; ++i; }
      const int jj = i + rem;
      double re = 0, im = 0;
      for (int w = 0; w < nw; ++w) { re += part[w][2 * q]; im += part[w][2 * q + 1]; }
      L[jj][i] = c128{re, -im};       // G[j][i] = conj(G[i][j]), lower triangle
    }
    __syncthreads();
    // G = L L^dag:  L[i][j] = (G[i][j] - sum_{k<j} L[i][k] conj(L[j][k])) / L[j][j], column by
    // column: the pivot by thread 0, then the rows below it, one thread each (every entry
    // accumulates over k in the same order as a serial loop would)
    for (int jj = 0; jj < Nv; ++jj) {
      if (t == 0) {
        const double gjj = L[jj][jj].re;
        double d = gjj;
        for (int k = 0; k < jj; ++k) d -= norm2(L[jj][k]);
        if (!(d > 1e-13 * gjj) || !(gjj > 0)) bad = 1;
        else L[jj][jj] = c128{sqrt(d), 0};
      }
      __syncthreads();
      if (bad) break;                  // the same for the whole workgroup
      const double ljj = L[jj][jj].re;
      for (int i = jj + 1 + t; i < Nv; i += blockDim.x) {
        c128 v = L[i][jj];
        for (int k = 0; k < jj; ++k) v = v - cmul_conj(L[jj][k], L[i][k]);
        L[i][jj] = (1.0 / ljj) * v;
      }
      __syncthreads();
    }
    __syncthreads();
    if (bad) break;                    // the same for the whole workgroup: keep the old block
    // P rows: p = w L^-dag  <=>  sum_{i<=j} p_i conj(L[j][i]) = w_j
    if (active) {
      for (int r = 0; r < 6; ++r) {
        // the row in registers: every index into pr is a compile-time constant
        // (the loops run to kMaxNv under conditions uniform across the wave)
        c128 pr[kMaxNv];
#pragma unroll
        for (int k = 0; k < kMaxNv; ++k) pr[k] = c128{0, 0};
        for (int jj = 0; jj < Nv; ++jj) {
          c128 v = field(jj)[(long long)(6 * h + r) * g.V + s];
#pragma unroll
          for (int i = 0; i < kMaxNv; ++i)
            if (i < jj) v = v - pr[i] * conj(L[jj][i]);
          const c128 pj = (1.0 / L[jj][jj].re) * v;
#pragma unroll
          for (int k = 0; k < kMaxNv; ++k)
            if (k == jj) pr[k] = pj;
        }
#pragma unroll
        for (int k = 0; k < kMaxNv; ++k)
          if (k < Nv) P[((long long)k * 12 + 6 * h + r) * g.V + s] = pr[k];
      }
    }
    __syncthreads();
  }
  if (t == 0 && bad) atomicOr(status, 1);
}

template <typename T>
__global__ void k_scatter_coarse(const cplx<T> *__restrict__ pc, int nf, const int *__restrict__ cols, int n2,
                                 int nA, cplx<T> *__restrict__ Qc) {
  // pc[j][d][A][row] -> Qc[A][d][row][cols[j]]
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long tot = (long long)nf * 5 * nA * n2;
  if (e >= tot) return;
  const int row = (int)(e % n2);
  long long r = e / n2;
  const int A = (int)(r % nA); r /= nA;
  const int d = (int)(r % 5);
  const int j = (int)(r / 5);
  Qc[(((long long)A * 5 + d) * n2 + row) * n2 + cols[j]] = pc[e];
}

}  // namespace

template <typename T>
void launch_restrict(const Geom &g, const cplx<T> *P, int Nv, const cplx<T> *f, long long fstride, int nf,
                     cplx<T> *c, hipStream_t st) {
  const int threads = ((g.bvol + 63) / 64) * 64;
  constexpr int R = transfer_group<T>();
  // algorithmic bytes: P once, the fields, the coarse output
  KTimerScope kt(KT_RESTRICT, ((double)g.V * 12.0 * (Nv + nf) + (double)nf * g.nblk * 2 * Nv) * sizeof(cplx<T>));
  LQ_LAUNCH(kt, (k_restrict<T, R>), dim3(g.nblk, (nf + R - 1) / R), dim3(threads), 0, st, g, P, Nv, f, fstride,
                     nf, c);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_prolong(const Geom &g, const cplx<T> *P, int Nv, const cplx<T> *c, cplx<T> *f, long long fstride,
                    int nf, bool accumulate, hipStream_t st) {
  const int threads = ((g.bvol + 63) / 64) * 64;
  constexpr int R = transfer_group<T>();
  // algorithmic bytes: P once, the coarse input, the fields out (and in when accumulating)
  KTimerScope kt(KT_PROLONG, ((double)g.V * 12.0 * (Nv + nf * (accumulate ? 2.0 : 1.0)) + (double)nf * g.nblk * 2 * Nv) *
                     sizeof(cplx<T>));
  LQ_LAUNCH(kt, (k_prolong<T, R>), dim3(g.nblk, (nf + R - 1) / R), dim3(threads), 0, st, g, P, Nv, c, f,
                     fstride, nf, accumulate);
  LQ_HIP(hipGetLastError());
}

void launch_build_P(const Geom &g, const c128 *const *cols, int Nv, c128 *P64, int *status, hipStream_t st) {
  const int threads = ((g.bvol + 63) / 64) * 64;
  hipLaunchKernelGGL(k_build_P, dim3(g.nblk, 2), dim3(threads), 0, st, g, cols, Nv, P64, status);
  LQ_HIP(hipGetLastError());
}

template <typename T>
void launch_scatter_coarse(const cplx<T> *parts_c, int nf, const int *cols_dev, int n2, int nA, cplx<T> *Qc,
                           hipStream_t st) {
  const long long tot = (long long)nf * 5 * nA * n2;
  hipLaunchKernelGGL((k_scatter_coarse<T>), dim3(blocks_for(tot, 256)), dim3(256), 0, st, parts_c, nf, cols_dev,
                     n2, nA, Qc);
  LQ_HIP(hipGetLastError());
}

#define LQ_INST(T)                                                                                           \
  template void launch_restrict<T>(const Geom &, const cplx<T> *, int, const cplx<T> *, long long, int,      \
                                   cplx<T> *, hipStream_t);                                                 \
  template void launch_prolong<T>(const Geom &, const cplx<T> *, int, const cplx<T> *, cplx<T> *, long long, \
                                  int, bool, hipStream_t);                                                  \
  template void launch_scatter_coarse<T>(const cplx<T> *, int, const int *, int, int, cplx<T> *, hipStream_t);
LQ_INST(float)
LQ_INST(double)
#undef LQ_INST

}  // namespace lq
