// Coarse-grid operator Q_c = P^dag Q P (sec. 2): a nearest-neighbour stencil
// on the lattice of aggregates with dense (2 Nv) x (2 Nv) complex blocks.
// Stored blocks per coarse site: the self block and the four forward blocks;
// the backward coupling from A - mu is the conjugate transpose of the
// forward block of A - mu, because Q_c is Hermitian.
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "lq_kernels.h"

namespace lq {
namespace {

__device__ inline int cnbr(const CoarseGeom &cg, int A, int mu, int step) {
  int a[4], r = A;
  for (int m = 0; m < 3; ++m) { a[m] = r % cg.nb[m]; r /= cg.nb[m]; }
  a[3] = r;
  a[mu] = (a[mu] + step + cg.nb[mu]) % cg.nb[mu];
  return a[0] + cg.nb[0] * (a[1] + cg.nb[1] * (a[2] + cg.nb[2] * a[3]));
}

// Block entries as read by the kernels: FP32/FP64 as stored, or bfloat16
// widened to FP32 (its bits are the upper half of the FP32 number).
template <typename T> __device__ inline cplx<T> qval(const cplx<T> &v) { return v; }
__device__ inline cplx<float> qval(const bf16c &v) {
  return mk<float>(__uint_as_float((unsigned)v.re << 16), __uint_as_float((unsigned)v.im << 16));
}

// FP32 -> bfloat16, round to nearest, ties to even; NaN stays NaN.
__device__ inline unsigned short to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__global__ void k_to_bf16(const cplx<float> *__restrict__ in, bf16c *__restrict__ out, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = bf16c{to_bf16(in[e].re), to_bf16(in[e].im)};
}

// One workgroup (one wave) per (coarse site, rhs); thread i computes row i.
template <typename T, typename QT>
__global__ void __launch_bounds__(64) k_coarse_apply(CoarseGeom cg, const QT *__restrict__ Qc,
                                                     const cplx<T> *__restrict__ xin, cplx<T> *__restrict__ yout,
                                                     Shifts sig, const double *__restrict__ dsig, bool g5form) {
  __shared__ cplx<T> xs[9][64];
  const int A = blockIdx.x, k = blockIdx.y, i = threadIdx.x;
  const int n2 = cg.n2;
  const cplx<T> *x = xin + (long long)k * cg.nA * n2;
  int nb[9];
  nb[0] = A;
  for (int mu = 0; mu < 4; ++mu) { nb[1 + mu] = cnbr(cg, A, mu, 1); nb[5 + mu] = cnbr(cg, A, mu, -1); }
  if (i < n2)
    for (int d = 0; d < 9; ++d) xs[d][i] = x[(long long)nb[d] * n2 + i];
  __syncthreads();
  if (i >= n2) return;
  const long long bs = (long long)n2 * n2;
  // self and forward blocks: row i of Qc[A][d]
  cplx<T> acc = mk<T>(0, 0);
  for (int d = 0; d < 5; ++d) {
    const QT *M = Qc + ((long long)A * 5 + d) * bs + (long long)i * n2;
    for (int j = 0; j < n2; ++j) acc = acc + qval(M[j]) * xs[d][j];
  }
  // backward: sum_j conj(Qc[A-mu][1+mu][j][i]) x_{A-mu}[j]
  for (int mu = 0; mu < 4; ++mu) {
    const QT *M = Qc + ((long long)nb[5 + mu] * 5 + 1 + mu) * bs + i;
    for (int j = 0; j < n2; ++j) acc = acc + cmul_conj(qval(M[(long long)j * n2]), xs[5 + mu][j]);
  }
  acc = acc - (T)(dsig ? dsig[k] : sig.s[k]) * xs[0][i];
  if (g5form && i >= n2 / 2) acc = -acc;
  yout[((long long)k * cg.nA + A) * n2 + i] = acc;
}

// All right-hand sides of one coarse site per workgroup: each (2Nv)^2 block is
// staged in LDS once and applied to every rhs, so the operator is read once
// per call instead of once per rhs.  Thread t owns row t % n2 for the rhs
// t / n2, t / n2 + 256 / n2, ...  The LDS rows are padded by one element, so
// threads reading the same column of different rows hit different banks, and
// the next block is loaded into registers while the current one is applied.
constexpr int kCoarseMaxN2 = 64;
constexpr int kCoarsePerThread = (kCoarseMaxN2 * kCoarseMaxN2 + 255) / 256;

template <typename T, typename QT, int KCH>
__global__ void __launch_bounds__(256) k_coarse_apply_multi(CoarseGeom cg, const QT *__restrict__ Qc,
                                                            const cplx<T> *__restrict__ xin,
                                                            cplx<T> *__restrict__ yout, Shifts sig,
                                                            const double *__restrict__ dsig, bool g5form, int nrhs) {
  __shared__ cplx<T> blk[kCoarseMaxN2 * (kCoarseMaxN2 + 1)];
  __shared__ cplx<T> xs[KCH][kCoarseMaxN2];
  const int A = blockIdx.x;
  const int n2 = cg.n2, ld = n2 + 1;
  const long long bs = (long long)n2 * n2;
  int nb[9];
  nb[0] = A;
  for (int mu = 0; mu < 4; ++mu) { nb[1 + mu] = cnbr(cg, A, mu, 1); nb[5 + mu] = cnbr(cg, A, mu, -1); }
  const int t = threadIdx.x;
  const int rows_per = n2;                          // threads per rhs
  const int rhs_slots = 256 / rows_per;             // rhs handled at once
  const int i = t % rows_per, ks = t / rows_per;
  auto block_ptr = [&](int d) -> const QT * {
    return (d < 5) ? Qc + ((long long)A * 5 + d) * bs : Qc + ((long long)nb[d] * 5 + (d - 4)) * bs;
  };
  // right-hand-side chunks of KCH: all of them in this workgroup, or with a
  // split grid (gridDim.y > 1) chunk y, y + gridDim.y, ...
  for (int k0 = blockIdx.y * KCH; k0 < nrhs; k0 += KCH * gridDim.y) {
    const int kc = (nrhs - k0 < KCH) ? nrhs - k0 : KCH;
    cplx<T> acc[(KCH + 3) / 4 > 0 ? (KCH + 3) / 4 : 1];
    const int nacc = (kc + rhs_slots - 1) / rhs_slots;
    for (int a = 0; a < (int)(sizeof(acc) / sizeof(acc[0])); ++a) acc[a] = mk<T>(0, 0);
    cplx<T> pre[kCoarsePerThread];
    {
      const QT *M = block_ptr(0);
#pragma unroll
      for (int q = 0; q < kCoarsePerThread; ++q) {
        const int e = t + 256 * q;
        pre[q] = (e < n2 * n2) ? qval(M[e]) : mk<T>(0, 0);
      }
    }
    for (int d = 0; d < 9; ++d) {
      __syncthreads();
#pragma unroll
      for (int q = 0; q < kCoarsePerThread; ++q) {
        const int e = t + 256 * q;
        if (e < n2 * n2) {
          const int r = e / n2, c = e - r * n2;
          blk[r * ld + c] = pre[q];
        }
      }
      for (int e = t; e < kc * n2; e += 256) {
        const int k = e / n2, j = e - k * n2;
        xs[k][j] = xin[((long long)(k0 + k) * cg.nA + nb[d]) * n2 + j];
      }
      __syncthreads();
      if (d + 1 < 9) {
        const QT *M = block_ptr(d + 1);
#pragma unroll
        for (int q = 0; q < kCoarsePerThread; ++q) {
          const int e = t + 256 * q;
          pre[q] = (e < n2 * n2) ? qval(M[e]) : mk<T>(0, 0);
        }
      }
      if (i < n2)
        for (int a = 0; a < nacc; ++a) {
          const int k = ks + a * rhs_slots;
          if (k >= kc) break;
          cplx<T> s = mk<T>(0, 0);
          if (d < 5)
            for (int j = 0; j < n2; ++j) s = s + blk[i * ld + j] * xs[k][j];
          else
            for (int j = 0; j < n2; ++j) s = s + cmul_conj(blk[j * ld + i], xs[k][j]);
          acc[a] = acc[a] + s;
        }
    }
    __syncthreads();
    if (i < n2 && ks < rhs_slots)
      for (int a = 0; a < nacc; ++a) {
        const int k = ks + a * rhs_slots;
        if (k >= kc) break;
        const long long off = ((long long)(k0 + k) * cg.nA + A) * n2 + i;
        cplx<T> v = acc[a] - (T)(dsig ? dsig[k0 + k] : sig.s[k0 + k]) * xin[off];
        if (g5form && i >= n2 / 2) v = -v;
        yout[off] = v;
      }
  }
}

// Matrix-core form (FP32 arithmetic; blocks stored in FP32 or bfloat16).  One
// workgroup per (coarse site, chunk of 16 right-hand sides) and one wave per
// 8 complex rows of the site's output, n2 / 8 waves.  For each of the nine
// couplings the 2Nv x 2Nv block and the neighbour's 16 vectors are staged in
// LDS (the next block is prefetched into registers meanwhile), and the complex
// product runs as real 16x16x4 MFMAs on an interleaved embedding: real row
// 2i + ri is (Re, Im) of complex row i, real k index 2j + kj is (Re, Im) of
// complex column j, so that
//   A[2i+ri][2j+kj] = Re M_ij (ri == kj), -Im M_ij (ri = 0, kj = 1), Im M_ij (ri = 1, kj = 0)
// for a stored block and the same with conj(M_ji) for a backward (conjugate
// transposed) one, and B[2j+kj][k] = (Re, Im) of x_k[j].  One MFMA consumes two
// complex columns; every multiply it does is a term of the complex product.
// Layouts of v_mfma_f32_16x16x4f32: lane l holds A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator register r of lane l is D[4 (l / 16) + r][l % 16].
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int kMfmaRhs = 16;
constexpr int kMfmaMaxN2 = 64;
constexpr int kMfmaPre = kMfmaMaxN2 / 8;     // block elements per thread: n2^2 / (8 n2)

template <typename QT>
__global__ void __launch_bounds__(512) k_coarse_apply_mfma(CoarseGeom cg, const QT *__restrict__ Qc,
                                                           const c64 *__restrict__ xin, c64 *__restrict__ yout,
                                                           Shifts sig, const double *__restrict__ dsig, bool g5form,
                                                           int nrhs) {
  __shared__ c64 blk[kMfmaMaxN2 * (kMfmaMaxN2 + 1)];
  __shared__ c64 xs[kMfmaMaxN2 * (kMfmaRhs + 1)];
  const int A = blockIdx.x, k0 = blockIdx.y * kMfmaRhs;
  const int n2 = cg.n2, ld = n2 + 1, ldx = kMfmaRhs + 1;
  const int kc = (nrhs - k0 < kMfmaRhs) ? nrhs - k0 : kMfmaRhs;
  const int t = threadIdx.x, nthr = blockDim.x;
  const int lane = t & 63, w = t >> 6;
  int nb[9];
  nb[0] = A;
  for (int mu = 0; mu < 4; ++mu) { nb[1 + mu] = cnbr(cg, A, mu, 1); nb[5 + mu] = cnbr(cg, A, mu, -1); }
  const long long bs = (long long)n2 * n2;
  auto block_ptr = [&](int d) -> const QT * {
    return (d < 5) ? Qc + ((long long)A * 5 + d) * bs : Qc + ((long long)nb[d] * 5 + (d - 4)) * bs;
  };
  // this lane's operand coordinates
  const int ci = 8 * w + ((lane & 15) >> 1), ri = lane & 1;     // A row: complex row, Re/Im
  const int kq = lane >> 4, kj = kq & 1;                      // k index in the step
  const int col = lane & 15;                                  // B / D column: right-hand side
  c64 pre[kMfmaPre];
#pragma unroll
  for (int q = 0; q < kMfmaPre; ++q) {
    const int e = t + nthr * q;
    pre[q] = (e < n2 * n2) ? qval(block_ptr(0)[e]) : mk<float>(0, 0);
  }
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 9; ++d) {
    __syncthreads();                                    // the previous block's reads are done
#pragma unroll
    for (int q = 0; q < kMfmaPre; ++q) {
      const int e = t + nthr * q;
      if (e < n2 * n2) blk[(e / n2) * ld + e % n2] = pre[q];
    }
    for (int e = t; e < kMfmaRhs * n2; e += nthr) {
      const int k = e / n2, j = e - k * n2;
      xs[j * ldx + k] = (k < kc) ? xin[((long long)(k0 + k) * cg.nA + nb[d]) * n2 + j] : mk<float>(0, 0);
    }
    __syncthreads();
    if (d + 1 < 9) {
      const QT *M = block_ptr(d + 1);
#pragma unroll
      for (int q = 0; q < kMfmaPre; ++q) {
        const int e = t + nthr * q;
        pre[q] = (e < n2 * n2) ? qval(M[e]) : mk<float>(0, 0);
      }
    }
    const bool back = d >= 5;
    for (int sstep = 0; sstep < n2 / 2; ++sstep) {
      const int cj = 2 * sstep + (kq >> 1);
      const c64 m = back ? blk[cj * ld + ci] : blk[ci * ld + cj];
      const float im = back ? -m.im : m.im;              // Im of the (i, j) entry
      const float a = (ri == kj) ? m.re : (ri ? im : -im);
      const c64 xv = xs[cj * ldx + col];
      const float b = kj ? xv.im : xv.re;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
  // lane holds complex rows 8w + 2 (l / 16) + h, h = 0, 1, of column col
  if (col < kc) {
    const float sg = (float)(dsig ? dsig[k0 + col] : sig.s[k0 + col]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int crow = 8 * w + 2 * kq + h;
      const long long off = ((long long)(k0 + col) * cg.nA + A) * n2 + crow;
      c64 v = mk<float>(acc[2 * h], acc[2 * h + 1]) - sg * xin[off];
      if (g5form && crow >= n2 / 2) v = -v;
      yout[off] = v;
    }
  }
}

// The same contraction on bfloat16 operands with FP32 accumulation
// (v_mfma_f32_16x16x16bf16_1k): the blocks as stored in bfloat16, the fields
// rounded to bfloat16 when staged.  Lane l holds A[l % 16][4 (l / 16) + i] and
// B[4 (l / 16) + i][l % 16], i = 0..3, and the accumulator layout of the FP32
// kernel above, so one MFMA covers 8 complex columns: in the interleaved
// embedding a lane's four k entries are (Re, Im) of two adjacent complex
// columns.  A 32-bit LDS word holds one complex entry (Re in the low half).
constexpr int kMfmaPre16 = kMfmaMaxN2 / 32;   // 16-byte block loads per thread: n2^2 / 4 / (8 n2)

__device__ inline unsigned bf16_pair(float re, float im) {
  return (unsigned)to_bf16(re) | ((unsigned)to_bf16(im) << 16);
}

__global__ void __launch_bounds__(512) k_coarse_apply_mfma_bf16(CoarseGeom cg, const bf16c *__restrict__ Qc,
                                                                const c64 *__restrict__ xin, c64 *__restrict__ yout,
                                                                Shifts sig, const double *__restrict__ dsig,
                                                                bool g5form, int nrhs) {
  typedef short v4s __attribute__((ext_vector_type(4)));
  __shared__ unsigned blk[kMfmaMaxN2 * (kMfmaMaxN2 + 1)];
  __shared__ unsigned xs[kMfmaMaxN2 * (kMfmaRhs + 1)];
  const int A = blockIdx.x, k0 = blockIdx.y * kMfmaRhs;
  const int n2 = cg.n2, ld = n2 + 1, ldx = kMfmaRhs + 1;
  const int kc = (nrhs - k0 < kMfmaRhs) ? nrhs - k0 : kMfmaRhs;
  const int t = threadIdx.x, nthr = blockDim.x;
  const int lane = t & 63, w = t >> 6;
  const int n16 = n2 * n2 / 4;                                 // 16-byte groups per block (n2 % 8 == 0)
  int nb[9];
  nb[0] = A;
  for (int mu = 0; mu < 4; ++mu) { nb[1 + mu] = cnbr(cg, A, mu, 1); nb[5 + mu] = cnbr(cg, A, mu, -1); }
  const long long bs = (long long)n2 * n2;
  auto block_ptr = [&](int d) -> const uint4 * {
    const bf16c *p = (d < 5) ? Qc + ((long long)A * 5 + d) * bs : Qc + ((long long)nb[d] * 5 + (d - 4)) * bs;
    return reinterpret_cast<const uint4 *>(p);
  };
  const int ci = 8 * w + ((lane & 15) >> 1), ri = lane & 1;    // A row: complex row, Re/Im
  const int kq = lane >> 4;                                   // columns 2 kq, 2 kq + 1 of each group of 8
  const int col = lane & 15;
  uint4 pre[kMfmaPre16];
#pragma unroll
  for (int q = 0; q < kMfmaPre16; ++q) {
    const int u = t + nthr * q;
    pre[q] = (u < n16) ? block_ptr(0)[u] : make_uint4(0, 0, 0, 0);
  }
  v4f acc = {0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < 9; ++d) {
    __syncthreads();                                    // the previous block's reads are done
#pragma unroll
    for (int q = 0; q < kMfmaPre16; ++q) {
      const int u = t + nthr * q;
      if (u < n16) {
        const int e = 4 * u, r = e / n2, cc = e - r * n2;         // 4 entries of one row
        unsigned *dst = blk + r * ld + cc;
        dst[0] = pre[q].x;
        dst[1] = pre[q].y;
        dst[2] = pre[q].z;
        dst[3] = pre[q].w;
      }
    }
    for (int e = t; e < kMfmaRhs * n2; e += nthr) {
      const int k = e / n2, j = e - k * n2;
      unsigned v = 0;
      if (k < kc) {
        const c64 xv = xin[((long long)(k0 + k) * cg.nA + nb[d]) * n2 + j];
        v = bf16_pair(xv.re, xv.im);
      }
      xs[j * ldx + k] = v;
    }
    __syncthreads();
    if (d + 1 < 9) {
      const uint4 *M = block_ptr(d + 1);
#pragma unroll
      for (int q = 0; q < kMfmaPre16; ++q) {
        const int u = t + nthr * q;
        pre[q] = (u < n16) ? M[u] : make_uint4(0, 0, 0, 0);
      }
    }
    // backward blocks are conjugate transposes: entry (i, j) = conj of stored (j, i)
    const bool back = d >= 5;
    const unsigned imflip = back ? 0x80000000u : 0u;
    for (int s = 0; s < n2 / 8; ++s) {
      const int cj = 8 * s + 2 * kq;
      unsigned m0 = back ? blk[cj * ld + ci] : blk[ci * ld + cj];
      unsigned m1 = back ? blk[(cj + 1) * ld + ci] : blk[ci * ld + cj + 1];
      m0 ^= imflip;
      m1 ^= imflip;
      // Re row: (Mr, -Mi); Im row: (Mi, Mr)
      const unsigned a0 = ri ? ((m0 >> 16) | (m0 << 16)) : (m0 ^ 0x80000000u);
      const unsigned a1 = ri ? ((m1 >> 16) | (m1 << 16)) : (m1 ^ 0x80000000u);
      const unsigned b0 = xs[cj * ldx + col], b1 = xs[(cj + 1) * ldx + col];
      v4s a, b;
      a[0] = (short)(a0 & 0xffffu); a[1] = (short)(a0 >> 16); a[2] = (short)(a1 & 0xffffu); a[3] = (short)(a1 >> 16);
      b[0] = (short)(b0 & 0xffffu); b[1] = (short)(b0 >> 16); b[2] = (short)(b1 & 0xffffu); b[3] = (short)(b1 >> 16);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
  }
  if (col < kc) {
    const float sg = (float)(dsig ? dsig[k0 + col] : sig.s[k0 + col]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int crow = 8 * w + 2 * kq + h;
      const long long off = ((long long)(k0 + col) * cg.nA + A) * n2 + crow;
      c64 v = mk<float>(acc[2 * h], acc[2 * h + 1]) - sg * xin[off];
      if (g5form && crow >= n2 / 2) v = -v;
      yout[off] = v;
    }
  }
}

template <typename T>
__global__ void k_coarse_g5(CoarseGeom cg, const cplx<T> *__restrict__ x, cplx<T> *__restrict__ y, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int i = (int)(e % cg.n2);
  const cplx<T> v = x[e];
  y[e] = (i >= cg.n2 / 2) ? -v : v;
}

__global__ void k_set_shifts(Shifts s, int n, double *dst) {
  const int k = threadIdx.x;
  if (k < n) dst[k] = s.s[k];
}

// Variants of the coarse apply: 0 = one wave per (site, rhs); 1..3 = one
// workgroup per site with the blocks staged in LDS for 4, 8 or 16 rhs per pass;
// 4, 5 = as 1, 2 with one workgroup per (site, chunk of 4 or 8 rhs), for
// coarse grids too small to fill the GPU with one workgroup per site; 6 = the
// matrix-core kernel (FP32 arithmetic only, 2Nv a multiple of 8 up to 64);
// 7 = the matrix-core kernel on bfloat16 operands (bfloat16 storage only, same
// block sizes; the fields are rounded to bfloat16 as well).
constexpr int kCoarseVariants = 8;
constexpr int kCoarseMfma = 6;
constexpr int kCoarseMfmaBf16 = 7;

template <typename T> bool mfma_applies(const CoarseGeom &cg) {
  return sizeof(T) == 4 && cg.n2 % 8 == 0 && cg.n2 <= kMfmaMaxN2;
}

template <typename T, typename QT> bool mfma_bf16_applies(const CoarseGeom &cg) {
  return std::is_same<QT, bf16c>::value && mfma_applies<T>(cg);
}

template <typename T, typename QT>
void coarse_launch_variant(int v, KTimerScope &kt, const CoarseGeom &cg, const QT *Qc, const cplx<T> *x,
                           cplx<T> *y, const Shifts &sig, const double *dsig, int nrhs, bool g5form, hipStream_t st) {
  switch (v) {
    case 1:
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 4>), dim3(cg.nA), dim3(256), 0, st, cg, Qc, x, y, sig, dsig, g5form,
                nrhs);
      break;
    case 2:
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 8>), dim3(cg.nA), dim3(256), 0, st, cg, Qc, x, y, sig, dsig, g5form,
                nrhs);
      break;
    case 3:
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 16>), dim3(cg.nA), dim3(256), 0, st, cg, Qc, x, y, sig, dsig,
                g5form, nrhs);
      break;
    case 4:
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 4>), dim3(cg.nA, (nrhs + 3) / 4), dim3(256), 0, st, cg, Qc, x, y,
                sig, dsig, g5form, nrhs);
      break;
    case 5:
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 8>), dim3(cg.nA, (nrhs + 7) / 8), dim3(256), 0, st, cg, Qc, x, y,
                sig, dsig, g5form, nrhs);
      break;
    case kCoarseMfmaBf16:
      if constexpr (std::is_same<T, float>::value && std::is_same<QT, bf16c>::value) {
        if (mfma_bf16_applies<T, QT>(cg)) {
          LQ_LAUNCH(kt, k_coarse_apply_mfma_bf16, dim3(cg.nA, (nrhs + kMfmaRhs - 1) / kMfmaRhs),
                    dim3(64 * (cg.n2 / 8)), 0, st, cg, Qc, x, y, sig, dsig, g5form, nrhs);
          break;
        }
      }
      // not applicable: as kernel 6
      [[fallthrough]];
    case kCoarseMfma:
      if constexpr (std::is_same<T, float>::value) {
        if (mfma_applies<T>(cg)) {
          LQ_LAUNCH(kt, (k_coarse_apply_mfma<QT>), dim3(cg.nA, (nrhs + kMfmaRhs - 1) / kMfmaRhs),
                    dim3(64 * (cg.n2 / 8)), 0, st, cg, Qc, x, y, sig, dsig, g5form, nrhs);
          break;
        }
      }
      // not applicable to this precision or block size: the LDS kernel for 8 rhs
      LQ_LAUNCH(kt, (k_coarse_apply_multi<T, QT, 8>), dim3(cg.nA), dim3(256), 0, st, cg, Qc, x, y, sig, dsig, g5form,
                nrhs);
      break;
    default:
      LQ_LAUNCH(kt, (k_coarse_apply<T, QT>), dim3(cg.nA, nrhs), dim3(64), 0, st, cg, Qc, x, y, sig, dsig, g5form);
  }
  LQ_HIP(hipGetLastError());
}

// The tuned variant per (arithmetic and storage precision, coarse sites, 2 Nv,
// nrhs, device).
struct CoarseTuneKey {
  int tsize, nA, n2, nrhs, dev;       // tsize: 100 * sizeof(T) + sizeof(QT)
  bool operator<(const CoarseTuneKey &o) const {
    return std::tie(tsize, nA, n2, nrhs, dev) < std::tie(o.tsize, o.nA, o.n2, o.nrhs, o.dev);
  }
};
std::mutex g_coarse_mu;
std::map<CoarseTuneKey, int> g_coarse_choice;
int g_coarse_force = -1;

CoarseTuneKey coarse_key(const CoarseGeom &cg, int tsize, int nrhs) {
  int dev = 0;
  LQ_HIP(hipGetDevice(&dev));
  return {tsize, cg.nA, cg.n2, nrhs, dev};
}

}  // namespace

int coarse_force_variant(int v) {
  if (v < -1 || v >= kCoarseVariants) return -1;
  std::lock_guard<std::mutex> lk(g_coarse_mu);
  g_coarse_force = v;
  return 0;
}

template <typename T, typename QT> int storage_code() { return 100 * (int)sizeof(T) + (int)sizeof(QT); }

template <typename T, typename QT>
int coarse_variant_q(const CoarseGeom &cg, int nrhs) {
  std::lock_guard<std::mutex> lk(g_coarse_mu);
  if (g_coarse_force >= 0) return g_coarse_force;
  auto it = g_coarse_choice.find(coarse_key(cg, storage_code<T, QT>(), nrhs));
  return it == g_coarse_choice.end() ? -1 : it->second;
}

template <typename T>
int coarse_variant(const CoarseGeom &cg, int nrhs) {
  return coarse_variant_q<T, cplx<T>>(cg, nrhs);
}

// Time every variant on the caller's operands (y is overwritten) and keep the
// fastest for this shape: one warm-up and three timed launches each, on the
// stream, outside any graph capture.  A shape already tuned is left alone.
template <typename T, typename QT>
int tune_coarse_apply_q(const CoarseGeom &cg, const QT *Qc, const cplx<T> *x, cplx<T> *y, int nrhs,
                        hipStream_t st) {
  const int known = coarse_variant_q<T, QT>(cg, nrhs);
  if (known >= 0) return known;
  Shifts z{};
  KTimerScope off(KT_COUNT, 0.0);     // never a selected class: untimed
  struct Events {                     // released on every exit, errors included
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  LQ_HIP(hipEventCreate(&ev.a));
  LQ_HIP(hipEventCreate(&ev.b));
  const hipEvent_t e0 = ev.a, e1 = ev.b;
  int best = 0;
  float tbest = 1e30f;
  for (int v = 0; v < kCoarseVariants; ++v) {
    if (v == kCoarseMfma && !mfma_applies<T>(cg)) continue;
    if (v == kCoarseMfmaBf16 && !mfma_bf16_applies<T, QT>(cg)) continue;
    coarse_launch_variant<T, QT>(v, off, cg, Qc, x, y, z, nullptr, nrhs, true, st);
    LQ_HIP(hipEventRecord(e0, st));
    for (int r = 0; r < 3; ++r) coarse_launch_variant<T, QT>(v, off, cg, Qc, x, y, z, nullptr, nrhs, true, st);
    LQ_HIP(hipEventRecord(e1, st));
    LQ_HIP(hipEventSynchronize(e1));
    float ms = 0;
    LQ_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (ms < tbest) { tbest = ms; best = v; }
  }
  std::lock_guard<std::mutex> lk(g_coarse_mu);
  g_coarse_choice[coarse_key(cg, storage_code<T, QT>(), nrhs)] = best;
  return best;
}

template <typename T>
int tune_coarse_apply(const CoarseGeom &cg, const cplx<T> *Qc, const cplx<T> *x, cplx<T> *y, int nrhs,
                      hipStream_t st) {
  return tune_coarse_apply_q<T, cplx<T>>(cg, Qc, x, y, nrhs, st);
}

int tune_coarse_apply_bf16(const CoarseGeom &cg, const bf16c *Qc, const c64 *x, c64 *y, int nrhs, hipStream_t st) {
  return tune_coarse_apply_q<float, bf16c>(cg, Qc, x, y, nrhs, st);
}

void launch_set_shifts(const Shifts &s, int n, double *dst, hipStream_t st) {
  hipLaunchKernelGGL(k_set_shifts, dim3(1), dim3(kMaxRhs), 0, st, s, n, dst);
  LQ_HIP(hipGetLastError());
}

void launch_to_bf16(const c64 *in, bf16c *out, long long n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(n, 256)), dim3(256), 0, st, in, out, n);
  LQ_HIP(hipGetLastError());
}

template <typename T, typename QT>
void coarse_apply_q(const CoarseGeom &cg, const QT *Qc, const cplx<T> *x, cplx<T> *y, const Shifts &sig, int nrhs,
                    bool g5form, hipStream_t st, const double *dsig) {
  // algorithmic bytes: the 5 stored blocks per site once, x in and y out per field
  KTimerScope kt(KT_COARSE, (double)cg.nA * 5 * cg.n2 * cg.n2 * sizeof(QT) +
                                2.0 * nrhs * cg.nA * cg.n2 * sizeof(cplx<T>));
  int v = coarse_variant_q<T, QT>(cg, nrhs);
  if (v < 0) {
    // untuned shape: few coarse sites (< 1024, e.g. 256 at 16^4 with 4^4
    // aggregates) keep one wave per (site, rhs); many sites stage each block
    // once for all rhs
    v = (nrhs >= 4 && cg.nA >= 1024) ? (sizeof(T) == 4 ? 3 : 2) : 0;
  }
  coarse_launch_variant<T, QT>(v, kt, cg, Qc, x, y, sig, dsig, nrhs, g5form, st);
}

template <typename T>
void launch_coarse_apply(const CoarseGeom &cg, const cplx<T> *Qc, const cplx<T> *x, cplx<T> *y, const Shifts &sig,
                         int nrhs, bool g5form, hipStream_t st, const double *dsig) {
  coarse_apply_q<T, cplx<T>>(cg, Qc, x, y, sig, nrhs, g5form, st, dsig);
}

void launch_coarse_apply_bf16(const CoarseGeom &cg, const bf16c *Qc, const c64 *x, c64 *y, const Shifts &sig,
                              int nrhs, bool g5form, hipStream_t st, const double *dsig) {
  coarse_apply_q<float, bf16c>(cg, Qc, x, y, sig, nrhs, g5form, st, dsig);
}

template <typename T>
void launch_coarse_g5(const CoarseGeom &cg, const cplx<T> *x, cplx<T> *y, int nrhs, hipStream_t st) {
  const long long n = (long long)nrhs * cg.nA * cg.n2;
  hipLaunchKernelGGL((k_coarse_g5<T>), dim3(blocks_for(n, 256)), dim3(256), 0, st, cg, x, y, n);
  LQ_HIP(hipGetLastError());
}

template void launch_coarse_apply<float>(const CoarseGeom &, const c64 *, const c64 *, c64 *, const Shifts &, int,
                                         bool, hipStream_t, const double *);
template void launch_coarse_apply<double>(const CoarseGeom &, const c128 *, const c128 *, c128 *, const Shifts &,
                                          int, bool, hipStream_t, const double *);
template int tune_coarse_apply<float>(const CoarseGeom &, const c64 *, const c64 *, c64 *, int, hipStream_t);
template int tune_coarse_apply<double>(const CoarseGeom &, const c128 *, const c128 *, c128 *, int, hipStream_t);
template int coarse_variant<float>(const CoarseGeom &, int);
template int coarse_variant<double>(const CoarseGeom &, int);
template void launch_coarse_g5<float>(const CoarseGeom &, const c64 *, c64 *, int, hipStream_t);
template void launch_coarse_g5<double>(const CoarseGeom &, const c128 *, c128 *, int, hipStream_t);

}  // namespace lq
