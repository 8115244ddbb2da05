// Products with a shared basis of long vectors (FP64): the Gram matrix
// C = E^dag W (nb basis vectors E_i against nw <= 16 vectors W_k) on the FP64
// matrix cores, and the combination U_k (+)= sum_i Y[i][k] E_i.  Both read
// every basis vector once per call.  They carry the Gram-Schmidt, Rayleigh-
// Ritz and Galerkin-correction products of the eigensolver.
//
// Gram kernel: split-K.  A workgroup owns a contiguous range of vector
// elements and has one wave per 16-row tile of E, so every wave does the same
// work; the W tile sits in LDS and is shared by all waves.  A complex inner
// product needs Re C = Er.Wr + Ei.Wi and Im C = Er.Wi - Ei.Wr.  Eight W
// vectors fill one 16-column MFMA operand as [Wr | Wi] and [Wi | -Wr]: two
// 16x16x4 FP64 MFMAs (A = Er, then A = Ei) leave [Re C | Im C] in one
// accumulator, so no MFMA work is spent on padding when nw <= 8.  Partial
// tiles go to scratch and a second kernel adds the chunks in a fixed order.
#include "lq_kernels.h"

namespace lq {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int kGramTile = 128;      // elements per LDS tile
constexpr int kGramMaxMT = 12;      // up to 192 basis vectors, one wave per 16-row tile
constexpr long long kGramMaxChunks = 2048;

template <int NCG>                   // column groups of 8 W vectors
__global__ void __launch_bounds__(64 * kGramMaxMT) k_gram(int nb, const c128 *__restrict__ E, long long estride,
                                                          int nw, const c128 *__restrict__ W, long long wstride,
                                                          long long n, long long per_chunk,
                                                          double *__restrict__ partial) {
  __shared__ c128 wt[8 * NCG][kGramTile + 4];     // +4: rows start on different LDS banks
  const int lane = threadIdx.x & 63, mt = threadIdx.x >> 6;
  const long long lo = (long long)blockIdx.x * per_chunk;
  const long long hi = (lo + per_chunk < n) ? lo + per_chunk : n;
  v4d acc[NCG];
#pragma unroll
  for (int g = 0; g < NCG; ++g) acc[g] = v4d{0, 0, 0, 0};
  // A operand: lane l holds A[l % 16][l / 16]: row = basis vector, k = element
  // B operand: lane l holds B[l / 16][l % 16]: k = element, column = (vector, part)
  // Rows past nb read row nb - 1 and their results are dropped; elements past
  // the chunk read its last element and meet zeros in the W tile.  The loads
  // are then unconditional and a wave keeps eight of them in flight.
  const int row = lane & 15, kk = lane >> 4;
  const int i = mt * 16 + row;
  const c128 *Ei = E + (long long)(i < nb ? i : nb - 1) * estride;
  const int wcol = lane & 7;
  const bool upper = (lane & 8) != 0;
  for (long long t0 = lo; t0 < hi; t0 += kGramTile) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < 8 * NCG * kGramTile; idx += blockDim.x) {
      const int k = idx / kGramTile, e = idx - k * kGramTile;
      const long long gi = t0 + e;
      wt[k][e] = (k < nw && gi < hi) ? W[(long long)k * wstride + gi] : c128{0, 0};
    }
    __syncthreads();
    const long long last = hi - 1 - t0;
    for (int s0 = 0; s0 < kGramTile / 4; s0 += 8) {
      c128 a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const long long e = 4 * (s0 + u) + kk;
        a[u] = Ei[t0 + (e < last ? e : last)];
      }
      // the scheduler otherwise sinks each load to its MFMA, one load in flight
#pragma unroll
      for (int u = 0; u < 8; ++u) asm volatile("" ::"v"(a[u].re), "v"(a[u].im));
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = 4 * (s0 + u) + kk;
#pragma unroll
        for (int g = 0; g < NCG; ++g) {
          const c128 w = wt[8 * g + wcol][e];
          const double b1 = upper ? w.im : w.re;
          const double b2 = upper ? -w.re : w.im;
          acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].re, b1, acc[g], 0, 0, 0);
          acc[g] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u].im, b2, acc[g], 0, 0, 0);
        }
      }
    }
  }
  // 16x16x4 FP64 MFMA result: register j of lane l holds D[4 j + l / 16][l % 16];
  // column c < 8 is Re C[., 8g + c], column c >= 8 is Im C[., 8g + c - 8]
#pragma unroll
  for (int g = 0; g < NCG; ++g) {
    const int k = 8 * g + wcol;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = mt * 16 + 4 * j + (lane >> 4);
      if (r < nb && k < nw) partial[(((long long)blockIdx.x * nb + r) * 16 + k) * 2 + (upper ? 1 : 0)] = acc[g][j];
    }
  }
}

// out[i][k] = sum over chunks of partial[chunk][i][k], fixed order.  One
// workgroup per row i: thread t adds column t % 16 over the chunks congruent
// to t / 16 modulo 16 (coalesced 256-byte rows of partials), then the 16
// group sums of a column are added in group order.
__global__ void __launch_bounds__(256) k_gram_final(int nb, int nw, int nchunks, const double *__restrict__ partial,
                                                    c128 *__restrict__ out) {
  __shared__ double red[16][16][2];
  const int i = blockIdx.x, t = threadIdx.x;
  const int k = t & 15, grp = t >> 4;
  double re = 0, im = 0;
  for (int c = grp; c < nchunks; c += 16) {
    const double *v = partial + (((long long)c * nb + i) * 16 + k) * 2;
    re += v[0];
    im += v[1];
  }
  red[grp][k][0] = re;
  red[grp][k][1] = im;
  __syncthreads();
  if (t < nw) {
    double sr = 0, si = 0;
    for (int g = 0; g < 16; ++g) { sr += red[g][t][0]; si += red[g][t][1]; }
    out[(long long)i * nw + t] = c128{sr, si};
  }
}

// U_k[e] = (U_k[e] if acc) + sum_i Y[i][k] E_i[e], one thread per element.
// The coefficients (up to 192 x 16, 48 KB) are the same for every thread: read
// from global memory by each wave they miss the scalar cache, so each
// workgroup stages them in LDS once (1.43x faster at 120 x 16).  E is read in
// batches of eight basis vectors with all loads in flight.
template <int NWT, bool EXACT>       // EXACT: nw == NWT, the column loop has no tests
__global__ void __launch_bounds__(256) k_combine(int nb, const c128 *__restrict__ E, long long estride, int nw,
                                                 const c128 *__restrict__ Y, c128 *__restrict__ U,
                                                 long long ustride, long long n, bool acc) {
  // every wave reads the same coefficient at a time (an LDS broadcast)
  extern __shared__ unsigned char comb_smem[];
  c128 *ys = reinterpret_cast<c128 *>(comb_smem);
  for (int q = threadIdx.x; q < nb * nw; q += blockDim.x) ys[q] = Y[q];
  __syncthreads();
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  c128 u[NWT];
#pragma unroll
  for (int k = 0; k < NWT; ++k) u[k] = c128{0, 0};
  const int nfull = nb & ~7;
  for (int i0 = 0; i0 < nfull; i0 += 8) {
    c128 v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = E[(long long)(i0 + q) * estride + e];
#pragma unroll
    for (int q = 0; q < 8; ++q) asm volatile("" ::"v"(v[q].re), "v"(v[q].im));
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const c128 *y = ys + (i0 + q) * nw;
#pragma unroll
      for (int k = 0; k < NWT; ++k)
        if (EXACT || k < nw) u[k] = u[k] + y[k] * v[q];
    }
  }
  for (int i = nfull; i < nb; ++i) {
    const c128 v = E[(long long)i * estride + e];
    const c128 *y = ys + i * nw;
#pragma unroll
    for (int k = 0; k < NWT; ++k)
      if (EXACT || k < nw) u[k] = u[k] + y[k] * v;
  }
#pragma unroll
  for (int k = 0; k < NWT; ++k)
    if (EXACT || k < nw) {
      c128 *p = U + (long long)k * ustride + e;
      *p = acc ? *p + u[k] : u[k];
    }
}

}  // namespace

size_t gram_scratch_elems(long long n) {
  (void)n;
  return (size_t)kGramMaxChunks * 192 * 16;
}

void launch_gram(int nb, const c128 *E, long long estride, int nw, const c128 *W, long long wstride, long long n,
                 c128 *out, c128 *scratch, hipStream_t st, long long max_chunks) {
  if (nb <= 0 || nw <= 0) return;
  if (nb > 16 * kGramMaxMT || nw > 16)
    throw HipError(hipErrorInvalidValue, "launch_gram: nb <= 192 and nw <= 16", __FILE__, __LINE__);
  if (max_chunks < 1) throw HipError(hipErrorInvalidValue, "launch_gram: max_chunks >= 1", __FILE__, __LINE__);
  // chunks of >= 1024 elements, enough of them to give every CU several
  // workgroups (16^4 fields: 768 chunks; 32^3 x 64: the 2048 maximum)
  long long nchunks = (n + 1023) / 1024;
  if (nchunks > kGramMaxChunks) nchunks = kGramMaxChunks;
  if (nchunks > max_chunks) nchunks = max_chunks;
  if (nchunks < 1) nchunks = 1;
  long long per = (n + nchunks - 1) / nchunks;
  per = ((per + kGramTile - 1) / kGramTile) * kGramTile;
  nchunks = (n + per - 1) / per;
  const int nmt = (nb + 15) / 16;
  double *part = reinterpret_cast<double *>(scratch);
  KTimerScope kt(KT_GRAM, (double)(nb + nw) * n * sizeof(c128));
  // timed from the start of the partial products to the end of the final sum
  const dim3 g1((unsigned)nchunks), b1(64 * nmt), g2(nb), b2(256);
  if (kt.on) {
    if (nw <= 8)
      hipExtLaunchKernelGGL((k_gram<1>), g1, b1, 0, st, kt.a, nullptr, 0, nb, E, estride, nw, W, wstride, n, per,
                            part);
    else
      hipExtLaunchKernelGGL((k_gram<2>), g1, b1, 0, st, kt.a, nullptr, 0, nb, E, estride, nw, W, wstride, n, per,
                            part);
    LQ_HIP(hipGetLastError());
    hipExtLaunchKernelGGL(k_gram_final, g2, b2, 0, st, nullptr, kt.b, 0, nb, nw, (int)nchunks, part, out);
  } else {
    if (nw <= 8)
      hipLaunchKernelGGL((k_gram<1>), g1, b1, 0, st, nb, E, estride, nw, W, wstride, n, per, part);
    else
      hipLaunchKernelGGL((k_gram<2>), g1, b1, 0, st, nb, E, estride, nw, W, wstride, n, per, part);
    LQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_gram_final, g2, b2, 0, st, nb, nw, (int)nchunks, part, out);
  }
  LQ_HIP(hipGetLastError());
}

void launch_combine(int nb, const c128 *E, long long estride, int nw, const c128 *Y, c128 *U, long long ustride,
                    long long n, bool accumulate, hipStream_t st) {
  if (nb <= 0 || nw <= 0) return;
  if (nb > 192 || nw > 16) throw HipError(hipErrorInvalidValue, "launch_combine: nb <= 192 and nw <= 16", __FILE__, __LINE__);
  const dim3 grid(blocks_for(n, 256)), block(256);
  KTimerScope kt(KT_COMBINE, (double)(nb + nw * (accumulate ? 2 : 1)) * n * sizeof(c128));
  const size_t shm = (size_t)nb * nw * sizeof(c128);
  if (nw == 8)
    LQ_LAUNCH(kt, (k_combine<8, true>), grid, block, shm, st, nb, E, estride, nw, Y, U, ustride, n, accumulate);
  else if (nw == 16)
    LQ_LAUNCH(kt, (k_combine<16, true>), grid, block, shm, st, nb, E, estride, nw, Y, U, ustride, n, accumulate);
  else if (nw < 8)
    LQ_LAUNCH(kt, (k_combine<8, false>), grid, block, shm, st, nb, E, estride, nw, Y, U, ustride, n, accumulate);
  else
    LQ_LAUNCH(kt, (k_combine<16, false>), grid, block, shm, st, nb, E, estride, nw, Y, U, ustride, n, accumulate);
  LQ_HIP(hipGetLastError());
}

}  // namespace lq

namespace lq {
namespace {

// out[t][i][k] = sum over the sites of timeslice t and the 12 components of
// conj(E_i) W_k, for canonical-layout fields [12][V] (t slowest, L3 sites per
// timeslice).  One workgroup per (t, i): its threads stride over the
// timeslice's 12 L3 entries with nw partial sums each, then a fixed-order
// reduction (wave shuffles, then the waves in order).
constexpr int kSliceMaxW = 16;
__global__ void __launch_bounds__(256) k_slice_products(int nb, const c128 *__restrict__ E, int nw,
                                                        const c128 *__restrict__ W, long long V, long long L3,
                                                        c128 *__restrict__ out) {
  __shared__ double red[4][kSliceMaxW][2];
  const int t = blockIdx.x, i = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double sr[kSliceMaxW], si[kSliceMaxW];
#pragma unroll
  for (int k = 0; k < kSliceMaxW; ++k) { sr[k] = 0; si[k] = 0; }
  const c128 *Ei = E + (long long)i * 12 * V;
  for (long long e = threadIdx.x; e < 12 * L3; e += blockDim.x) {
    const long long c = e / L3, x = t * L3 + (e - c * L3);
    const c128 a = Ei[c * V + x];
#pragma unroll
    for (int k = 0; k < kSliceMaxW; ++k) {
      if (k >= nw) break;
      const c128 b = W[(long long)k * 12 * V + c * V + x];
      sr[k] += a.re * b.re + a.im * b.im;
      si[k] += a.re * b.im - a.im * b.re;
    }
  }
#pragma unroll
  for (int k = 0; k < kSliceMaxW; ++k) {
    for (int off = 32; off > 0; off >>= 1) {
      sr[k] += __shfl_xor(sr[k], off, 64);
      si[k] += __shfl_xor(si[k], off, 64);
    }
    if (lane == 0) { red[wave][k][0] = sr[k]; red[wave][k][1] = si[k]; }
  }
  __syncthreads();
  if (threadIdx.x < nw) {
    const int k = threadIdx.x;
    double a = 0, b = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { a += red[w][k][0]; b += red[w][k][1]; }
    out[((long long)t * nb + i) * nw + k] = c128{a, b};
  }
}

}  // namespace

void launch_slice_products(int nb, const c128 *E, int nw, const c128 *W, long long V, int T, c128 *out,
                           hipStream_t st) {
  if (nb < 1 || nw < 1 || nw > kSliceMaxW || T < 1 || V % T)
    throw HipError(hipErrorInvalidValue, "launch_slice_products: nw <= 16, T divides V", __FILE__, __LINE__);
  hipLaunchKernelGGL(k_slice_products, dim3(T, nb), dim3(256), 0, st, nb, E, nw, W, V, V / T, out);
  LQ_HIP(hipGetLastError());
}

}  // namespace lq
