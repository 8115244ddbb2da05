// Products with a shared basis of long vectors (FP64): the Gram matrix
// C = E^dag W (nb basis vectors E_i against nw <= 16 vectors W_k) on the FP64
// matrix cores, and the combination U_k (+)= sum_i Y[i][k] E_i.  Both read
// every basis vector once per call.  They carry the Gram-Schmidt, Rayleigh-
// Ritz and Galerkin-correction products of the eigensolver.
//
// Gram kernel: split-K.  A workgroup owns a contiguous range of vector
// elements; it stages the W tile (16 x 64 elements) in LDS and its four waves
// run 16x16x4 FP64 MFMAs over 16-row tiles of E.  A complex inner product is
// four real products: Re C = Er.Wr + Ei.Wi, Im C = Er.Wi - Ei.Wr.  Partial
// tiles go to scratch and a second kernel adds the chunks in a fixed order.
#include "lq_kernels.h"

namespace lq {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramTile = 64;       // elements per LDS tile
constexpr int kGramMaxMT = 10;      // up to 160 basis vectors

__global__ void __launch_bounds__(256) k_gram(int nb, const c128 *__restrict__ E, long long estride, int nw,
                                              const c128 *__restrict__ W, long long wstride, long long n,
                                              long long per_chunk, c128 *__restrict__ partial) {
  __shared__ c128 wt[16][kGramTile];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long long lo = (long long)blockIdx.x * per_chunk;
  const long long hi = (lo + per_chunk < n) ? lo + per_chunk : n;
  const int nmt = (nb + 15) / 16;
  v4d acc_re[3], acc_im[3];          // up to 3 M-tiles per wave (nb <= 192)
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    acc_re[q] = v4d{0, 0, 0, 0};
    acc_im[q] = v4d{0, 0, 0, 0};
  }
  const int row = lane & 15, kk = lane >> 4;
  for (long long t0 = lo; t0 < hi; t0 += kGramTile) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 16 * kGramTile; idx += 256) {
      const int k = idx / kGramTile, e = idx - k * kGramTile;
      const long long g = t0 + e;
      wt[k][e] = (k < nw && g < hi) ? W[(long long)k * wstride + g] : c128{0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int mt = wave + 4 * q;
      if (mt >= nmt) break;
      const int i = mt * 16 + row;
      const c128 *Ei = E + (long long)i * estride;
#pragma unroll 4
      for (int s = 0; s < kGramTile / 4; ++s) {
        const int e = 4 * s + kk;
        const long long g = t0 + e;
        c128 a = (i < nb && g < hi) ? Ei[g] : c128{0, 0};
        const c128 b = wt[row][e];          // B[k = e][col = row] -> W_row[e]
        acc_re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.re, acc_re[q], 0, 0, 0);
        acc_re[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.im, b.im, acc_re[q], 0, 0, 0);
        acc_im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.re, b.im, acc_im[q], 0, 0, 0);
        acc_im[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.im, b.re, acc_im[q], 0, 0, 0);
      }
    }
  }
  // 16x16x4 FP64 MFMA result: register j of lane l holds D[4 j + l / 16][l % 16]
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int mt = wave + 4 * q;
    if (mt >= nmt) break;
    const int col = lane & 15;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 4 * j + (lane >> 4);
      const int i = mt * 16 + r;
      if (i < nb && col < nw)
        partial[((long long)blockIdx.x * nb + i) * 16 + col] = c128{acc_re[q][j], acc_im[q][j]};
    }
  }
}

// out[i][k] = sum over chunks of partial[chunk][i][k], fixed order
__global__ void k_gram_final(int nb, int nw, int nchunks, const c128 *__restrict__ partial, c128 *__restrict__ out) {
  const int ik = blockIdx.x * blockDim.x + threadIdx.x;
  if (ik >= nb * nw) return;
  const int i = ik / nw, k = ik - i * nw;
  double re = 0, im = 0;
  for (int c = 0; c < nchunks; ++c) {
    const c128 v = partial[((long long)c * nb + i) * 16 + k];
    re += v.re;
    im += v.im;
  }
  out[ik] = c128{re, im};
}

// U_k[e] = (U_k[e] if acc) + sum_i Y[i][k] E_i[e], one thread per element
__global__ void __launch_bounds__(256) k_combine(int nb, const c128 *__restrict__ E, long long estride, int nw,
                                                 const c128 *__restrict__ Y, c128 *__restrict__ U,
                                                 long long ustride, long long n, bool acc) {
  extern __shared__ c128 ys[];        // [nb][nw]
  for (int idx = threadIdx.x; idx < nb * nw; idx += blockDim.x) ys[idx] = Y[idx];
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  c128 u[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) u[k] = c128{0, 0};
  for (int i = 0; i < nb; ++i) {
    const c128 v = E[(long long)i * estride + e];
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < nw) u[k] = u[k] + ys[i * nw + k] * v;
  }
#pragma unroll
  for (int k = 0; k < 16; ++k)
    if (k < nw) {
      c128 *p = U + (long long)k * ustride + e;
      *p = acc ? *p + u[k] : u[k];
    }
}

}  // namespace

size_t gram_scratch_elems(long long n) {
  (void)n;
  return (size_t)1024 * 192 * 16;
}

void launch_gram(int nb, const c128 *E, long long estride, int nw, const c128 *W, long long wstride, long long n,
                 c128 *out, c128 *scratch, hipStream_t st) {
  if (nb <= 0 || nw <= 0) return;
  if (nb > 192 || nw > 16) throw HipError(hipErrorInvalidValue, "launch_gram: nb <= 192 and nw <= 16", __FILE__, __LINE__);
  long long nchunks = (n + 4095) / 4096;
  if (nchunks > 1024) nchunks = 1024;
  if (nchunks < 1) nchunks = 1;
  long long per = (n + nchunks - 1) / nchunks;
  per = ((per + kGramTile - 1) / kGramTile) * kGramTile;
  nchunks = (n + per - 1) / per;
  hipLaunchKernelGGL(k_gram, dim3((unsigned)nchunks), dim3(256), 0, st, nb, E, estride, nw, W, wstride, n, per,
                     scratch);
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_gram_final, dim3(blocks_for((long long)nb * nw, 256)), dim3(256), 0, st, nb, nw,
                     (int)nchunks, scratch, out);
  LQ_HIP(hipGetLastError());
}

void launch_combine(int nb, const c128 *E, long long estride, int nw, const c128 *Y, c128 *U, long long ustride,
                    long long n, bool accumulate, hipStream_t st) {
  if (nb <= 0 || nw <= 0) return;
  if (nb > 192 || nw > 16) throw HipError(hipErrorInvalidValue, "launch_combine: nb <= 192 and nw <= 16", __FILE__, __LINE__);
  const size_t lds = (size_t)nb * nw * sizeof(c128);
  hipLaunchKernelGGL(k_combine, dim3(blocks_for(n, 256)), dim3(256), lds, st, nb, E, estride, nw, Y, U, ustride, n,
                     accumulate);
  LQ_HIP(hipGetLastError());
}

}  // namespace lq
