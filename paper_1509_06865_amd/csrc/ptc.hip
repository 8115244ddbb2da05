// Parallel-transport convolution: the layer of the network that proposes
// multigrid test vectors for the learned setup (not part of the paper).
//
//   out[o](x) = sum_i sum_{d in {-1,0,1}^4} W[o][i][d] T_d(x) phi[i](x + d)
//
// W[o][i][d] is a 4x4 complex matrix on spin; T_d(x) the 3x3 colour matrix
// given by the product of the links along the path from x to x + d that steps
// through the directions 0, 1, 2, 3 in that order: U_mu(y) for a step +mu from
// y, U_mu(y - mu)^dag for a step -mu, times the boundary sign for a step across
// the t boundary.  Offsets are numbered k = sum_mu (d_mu + 1) 3^(3 - mu).
//
// This is the direct form: one thread per (site, output channel), the path
// products formed on the fly, FP64.  It is the correctness reference on the
// device for the GEMM-shaped (MFMA) form the layer takes at scale.
#include <algorithm>
#include "lq_kernels.h"
#include "lq_dslash.h"

namespace lq {
namespace {

constexpr int kPtcOffsets = 81;

__device__ inline void mat3_mul(const c128 A[9], const c128 B[9], c128 C[9]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) C[3 * a + b] = A[3 * a] * B[b] + A[3 * a + 1] * B[3 + b] + A[3 * a + 2] * B[6 + b];
}

__device__ inline void offset_of(int k, int d[4]) {
  for (int mu = 3; mu >= 0; --mu) { d[mu] = k % 3 - 1; k /= 3; }
}

// T_d(x): the links along the path from x to x + d (directions 0..3 in order,
// boundary signs included); returns the site x + d.
__device__ inline int path_transport(const Geom &g, const c128 *__restrict__ U, int x, const int d[4], c128 T[9]) {
  const long long V = g.V;
#pragma unroll
  for (int e = 0; e < 9; ++e) T[e] = c128{(e % 4 == 0) ? 1.0 : 0.0, 0};
  int pos = x;
  for (int mu = 0; mu < 4; ++mu) {
    if (d[mu] == 0) continue;
    const SiteCoord c = decode(g, pos);
    float sg;
    bool in;
    c128 L[9], P[9];
    if (d[mu] > 0) {
      const int nxt = neighbour(g, pos, c, mu, true, &sg, &in);
      load_link(U, V, mu, pos, L);
      pos = nxt;
    } else {
      const int nxt = neighbour(g, pos, c, mu, false, &sg, &in);
      c128 M[9];
      load_link(U, V, mu, nxt, M);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) L[3 * a + b] = conj(M[3 * b + a]);
      pos = nxt;
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) L[e] = (double)sg * L[e];
    mat3_mul(T, L, P);
#pragma unroll
    for (int e = 0; e < 9; ++e) T[e] = P[e];
  }
  return pos;
}

// the site x - d (the start of the path that ends at y)
__device__ inline int back_offset(const Geom &g, int y, const int d[4]) {
  int pos = y;
  for (int mu = 0; mu < 4; ++mu) {
    if (d[mu] == 0) continue;
    float sg;
    bool in;
    pos = neighbour(g, pos, decode(g, pos), mu, d[mu] < 0, &sg, &in);
  }
  return pos;
}

__global__ void __launch_bounds__(256) k_ptc_forward(Geom g, const c128 *__restrict__ U, int cin,
                                                     const c128 *__restrict__ phi, const c128 *__restrict__ W,
                                                     c128 *__restrict__ out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= g.V) return;
  const int o = blockIdx.y;
  const long long V = g.V;
  c128 acc[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) acc[e] = c128{0, 0};
  for (int k = 0; k < kPtcOffsets; ++k) {
    int d[4];
    offset_of(k, d);
    c128 T[9];
    const int pos = path_transport(g, U, x, d, T);       // T_d(x) and x + d
    for (int i = 0; i < cin; ++i) {
      c128 p[12], q[12];
      load_spinor(phi + (long long)i * 12 * V, V, pos, p);
      // colour: q[s][a] = sum_b T[a][b] p[s][b]
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          q[3 * s + a] = T[3 * a] * p[3 * s] + T[3 * a + 1] * p[3 * s + 1] + T[3 * a + 2] * p[3 * s + 2];
      // spin: acc[s][a] += sum_t W[o][i][k][s][t] q[t][a]
      const c128 *w = W + (((long long)o * cin + i) * kPtcOffsets + k) * 16;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        const c128 w0 = w[4 * s], w1 = w[4 * s + 1], w2 = w[4 * s + 2], w3 = w[4 * s + 3];
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[3 * s + a] = acc[3 * s + a] + w0 * q[a] + w1 * q[3 + a] + w2 * q[6 + a] + w3 * q[9 + a];
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 12; ++e) out[((long long)o * 12 + e) * V + x] = acc[e];
}

// Gradients, for a real loss L and g = dL/dRe(out) + i dL/dIm(out) (so that
// dL = Re sum conj(g) d(out)); the results have the same form for phi and W.
// Input gradient, one thread per (site y, input channel i):
//   g_in[i](y) = sum_o sum_d W[o][i][d]^dag T_d(y - d)^dag g[o](y - d).
__global__ void __launch_bounds__(256) k_ptc_grad_input(Geom g, const c128 *__restrict__ U, int cout,
                                                        const c128 *__restrict__ gout, int cin,
                                                        const c128 *__restrict__ W, c128 *__restrict__ gin) {
  const int y = blockIdx.x * blockDim.x + threadIdx.x;
  if (y >= g.V) return;
  const int i = blockIdx.y;
  const long long V = g.V;
  c128 acc[12];
#pragma unroll
  for (int e = 0; e < 12; ++e) acc[e] = c128{0, 0};
  for (int k = 0; k < kPtcOffsets; ++k) {
    int d[4];
    offset_of(k, d);
    const int x = back_offset(g, y, d);
    c128 T[9];
    (void)path_transport(g, U, x, d, T);              // ends at y
    for (int o = 0; o < cout; ++o) {
      c128 p[12], q[12];
      load_spinor(gout + (long long)o * 12 * V, V, x, p);
      // colour: q[s][a] = sum_b conj(T[b][a]) p[s][b]
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          q[3 * s + a] = cmul_conj(T[a], p[3 * s]) + cmul_conj(T[3 + a], p[3 * s + 1]) + cmul_conj(T[6 + a], p[3 * s + 2]);
      // spin: acc[t][a] += sum_s conj(W[s][t]) q[s][a]
      const c128 *w = W + (((long long)o * cin + i) * kPtcOffsets + k) * 16;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const c128 w0 = w[t], w1 = w[4 + t], w2 = w[8 + t], w3 = w[12 + t];
#pragma unroll
        for (int a = 0; a < 3; ++a)
          acc[3 * t + a] = acc[3 * t + a] + cmul_conj(w0, q[a]) + cmul_conj(w1, q[3 + a]) + cmul_conj(w2, q[6 + a]) +
                           cmul_conj(w3, q[9 + a]);
      }
    }
  }
#pragma unroll
  for (int e = 0; e < 12; ++e) gin[((long long)i * 12 + e) * V + y] = acc[e];
}

// Weight gradient, one workgroup per (o, i, d), sites summed in a fixed order:
//   g_W[o][i][d][s][t] = sum_x sum_a g[o](x)[s][a] conj((T_d(x) phi[i](x + d))[t][a]).
__global__ void __launch_bounds__(256) k_ptc_grad_weight(Geom g, const c128 *__restrict__ U, int cin,
                                                         const c128 *__restrict__ phi, int cout,
                                                         const c128 *__restrict__ gout, c128 *__restrict__ gW) {
  __shared__ double red[4][32];
  const int k = blockIdx.x % kPtcOffsets;
  const int oi = blockIdx.x / kPtcOffsets;
  const int i = oi % cin, o = oi / cin;
  const long long V = g.V;
  int d[4];
  offset_of(k, d);
  double pr[16], pi[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) { pr[e] = 0; pi[e] = 0; }
  for (int x = threadIdx.x; x < g.V; x += blockDim.x) {
    c128 T[9], p[12], tp[12], gg[12];
    const int pos = path_transport(g, U, x, d, T);
    load_spinor(phi + (long long)i * 12 * V, V, pos, p);
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int a = 0; a < 3; ++a)
        tp[3 * t + a] = T[3 * a] * p[3 * t] + T[3 * a + 1] * p[3 * t + 1] + T[3 * a + 2] * p[3 * t + 2];
    load_spinor(gout + (long long)o * 12 * V, V, x, gg);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        c128 v = c128{0, 0};
#pragma unroll
        for (int a = 0; a < 3; ++a) v = v + cmul_conj(tp[3 * t + a], gg[3 * s + a]);   // gg * conj(tp)
        pr[4 * s + t] += v.re;
        pi[4 * s + t] += v.im;
      }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int e = 0; e < 16; ++e) {
    double re = pr[e], im = pi[e];
    for (int off = 32; off > 0; off >>= 1) {
      re += __shfl_xor(re, off, 64);
      im += __shfl_xor(im, off, 64);
    }
    if (lane == 0) { red[wave][2 * e] = re; red[wave][2 * e + 1] = im; }
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int e = threadIdx.x;
    double re = 0, im = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) { re += red[w][2 * e]; im += red[w][2 * e + 1]; }
    gW[(long long)blockIdx.x * 16 + e] = c128{re, im};
  }
}

// phi -> phi * relu(|phi(x)| + b[c]) / |phi(x)| for channel c at site x, with
// |phi(x)| the norm over the 12 spin-colour components (0 where it vanishes).
// One thread per (site, channel); out may be phi.
// out may be phi (each thread reads its site's 12 components before writing
// them), so phi and out are not marked restrict
__global__ void __launch_bounds__(256) k_mod_relu(int V, const c128 *phi, const double *__restrict__ b,
                                                  c128 *out) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  const int ch = blockIdx.y;
  const c128 *p = phi + (long long)ch * 12 * V + x;
  c128 v[12];
  double n2 = 0;
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    v[e] = p[(long long)e * V];
    n2 += v[e].re * v[e].re + v[e].im * v[e].im;
  }
  const double n = sqrt(n2);
  const double scale = (n > 0) ? fmax(n + b[ch], 0.0) / n : 0.0;
  c128 *q = out + (long long)ch * 12 * V + x;
#pragma unroll
  for (int e = 0; e < 12; ++e) q[(long long)e * V] = scale * v[e];
}

// Gradients through the nonlinearity (same convention as the layer's): with
// n = |phi(x)| and s = relu(n + b) / n, where n + b > 0
//   g_phi = s g - (b / n^3) Re<g, phi> phi,   contrib(x) = Re<g, phi> / n,
// and 0 elsewhere; g_b[c] = sum_x contrib(x) (k_sum_rows).
__global__ void __launch_bounds__(256) k_mod_relu_grad(int V, const c128 *__restrict__ phi,
                                                       const double *__restrict__ b, const c128 *__restrict__ gout,
                                                       c128 *__restrict__ gphi, double *__restrict__ contrib) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= V) return;
  const int ch = blockIdx.y;
  const long long base = (long long)ch * 12 * V + x;
  c128 v[12], gg[12];
  double n2 = 0, gp = 0;                               // |phi|^2, Re<g, phi>
#pragma unroll
  for (int e = 0; e < 12; ++e) {
    v[e] = phi[base + (long long)e * V];
    gg[e] = gout[base + (long long)e * V];
    n2 += v[e].re * v[e].re + v[e].im * v[e].im;
    gp += gg[e].re * v[e].re + gg[e].im * v[e].im;
  }
  const double n = sqrt(n2);
  const bool on = n > 0 && n + b[ch] > 0;
  const double sc = on ? (n + b[ch]) / n : 0.0;
  const double cphi = on ? -b[ch] * gp / (n2 * n) : 0.0;
#pragma unroll
  for (int e = 0; e < 12; ++e) gphi[base + (long long)e * V] = sc * gg[e] + cphi * v[e];
  contrib[(long long)ch * V + x] = on ? gp / n : 0.0;
}

// out[r] = sum_x a[r][x], one workgroup per row, fixed order (strided
// partial sums, then a shuffle tree and the waves in order).
__global__ void __launch_bounds__(256) k_sum_rows(int V, const double *__restrict__ a, double *__restrict__ out) {
  __shared__ double red[4];
  const int r = blockIdx.x;
  double v = 0;
  for (int x = threadIdx.x; x < V; x += blockDim.x) v += a[(long long)r * V + x];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    out[r] = t;
  }
}

// Training loss of the network's outputs X ([n_out][12][V]) for targets u
// ([K][12][V]), canonical layout: for each aggregate A (extents agg) and gamma5
// half h, with M the (6|A|) x n_out rows of X and B those of u,
//   coef = (M^dag M)^-1 M^dag B,  R = B - M coef,
//   loss part = sum |R|^2 / K,  gradient rows = -(2/K) R coef^dag
// (the gradient in the same form as the layer's).  One workgroup per (A, h);
// G = M^dag M and C = M^dag B accumulate over the rows, thread 0 solves with
// Cholesky in LDS.  A pivot at or below 1e-13 of its diagonal entry (outputs
// dependent, or nearly so, on the block) raises *status.
constexpr int kProjMax = 32;

__device__ inline int proj_site(const int L[4], const int agg[4], int blk, int loc) {
  int x[4];
  for (int m = 0; m < 4; ++m) {
    const int nb = L[m] / agg[m];
    const int a = blk % nb, l = loc % agg[m];
    blk /= nb;
    loc /= agg[m];
    x[m] = a * agg[m] + l;
  }
  return x[0] + L[0] * (x[1] + L[1] * (x[2] + L[2] * x[3]));
}

struct ProjGeom { int L[4]; int agg[4]; int bvol; int V; };

__global__ void __launch_bounds__(256) k_proj_loss(ProjGeom pg, int nout, const c128 *__restrict__ X, int K,
                                                   const c128 *__restrict__ u, double *__restrict__ part,
                                                   c128 *__restrict__ gX, int *__restrict__ status) {
  __shared__ c128 G[kProjMax][kProjMax];
  __shared__ c128 C[kProjMax][kProjMax];
  __shared__ double red[4];
  __shared__ int bad;
  const int blk = blockIdx.x >> 1, h = blockIdx.x & 1;
  const int rows = 6 * pg.bvol;
  const long long V = pg.V;
  if (threadIdx.x == 0) bad = 0;
  // row r: component 6h + r / bvol at the site of local index r % bvol
  auto at = [&](const c128 *F, int col, int r) -> c128 {
    const int comp = 6 * h + r / pg.bvol, site = proj_site(pg.L, pg.agg, blk, r % pg.bvol);
    return F[((long long)col * 12 + comp) * V + site];
  };
  for (int e = threadIdx.x; e < nout * nout + nout * K; e += blockDim.x) {
    const bool isG = e < nout * nout;
    const int p = isG ? e / nout : (e - nout * nout) / K;
    const int q = isG ? e % nout : (e - nout * nout) % K;
    c128 acc = c128{0, 0};
    for (int r = 0; r < rows; ++r) acc = acc + cmul_conj(at(X, p, r), isG ? at(X, q, r) : at(u, q, r));
    if (isG) G[p][q] = acc; else C[p][q] = acc;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // G = L L^dag in place (lower triangle), then coef = G^-1 C into C
    for (int j = 0; j < nout; ++j) {
      // the same relative pivot test as the setup's local orthonormalisation:
      // outputs that are dependent, or nearly so, on the block are rejected
      const double gjj = G[j][j].re;
      double dj = gjj;
      for (int k = 0; k < j; ++k) dj -= G[j][k].re * G[j][k].re + G[j][k].im * G[j][k].im;
      if (!(dj > 1e-13 * gjj) || !(gjj > 0)) { bad = 1; dj = 1.0; }
      const double ljj = sqrt(dj);
      G[j][j] = c128{ljj, 0};
      for (int i = j + 1; i < nout; ++i) {
        c128 v = G[i][j];
        for (int k = 0; k < j; ++k) v = v - G[i][k] * conj(G[j][k]);
        G[i][j] = (1.0 / ljj) * v;
      }
    }
    for (int k = 0; k < K; ++k) {
      for (int i = 0; i < nout; ++i) {                // L y = c
        c128 v = C[i][k];
        for (int j = 0; j < i; ++j) v = v - G[i][j] * C[j][k];
        C[i][k] = (1.0 / G[i][i].re) * v;
      }
      for (int i = nout - 1; i >= 0; --i) {           // L^dag x = y
        c128 v = C[i][k];
        for (int j = i + 1; j < nout; ++j) v = v - cmul_conj(G[j][i], C[j][k]);
        C[i][k] = (1.0 / G[i][i].re) * v;
      }
    }
  }
  __syncthreads();
  double lp = 0;
  for (int r = threadIdx.x; r < rows; r += blockDim.x) {
    c128 R[kProjMax];
    for (int k = 0; k < K; ++k) {
      c128 v = at(u, k, r);
      for (int p = 0; p < nout; ++p) v = v - at(X, p, r) * C[p][k];
      R[k] = v;
      lp += v.re * v.re + v.im * v.im;
    }
    if (gX) {
      const int comp = 6 * h + r / pg.bvol, site = proj_site(pg.L, pg.agg, blk, r % pg.bvol);
      for (int p = 0; p < nout; ++p) {
        c128 gsum = c128{0, 0};
        for (int k = 0; k < K; ++k) gsum = gsum + R[k] * conj(C[p][k]);
        gX[((long long)p * 12 + comp) * V + site] = (-2.0 / K) * gsum;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) lp += __shfl_xor(lp, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lp;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    part[blockIdx.x] = t / K;
    if (bad) atomicOr(status, 1);
  }
}

// One Adam step on n real values (a complex parameter is its real and
// imaginary parts):  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
// p -= (lr / bc1) m / (sqrt(v) / sqrt(bc2) + eps),  bc_i = 1 - b_i^t.
__global__ void k_adam(long long n, double *__restrict__ p, const double *__restrict__ g, double *__restrict__ m,
                       double *__restrict__ v, double lr, double b1, double b2, double eps, double bc1,
                       double sbc2) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const double gi = g[e];
  const double mi = b1 * m[e] + (1.0 - b1) * gi;
  const double vi = b2 * v[e] + (1.0 - b2) * gi * gi;
  m[e] = mi;
  v[e] = vi;
  p[e] -= (lr / bc1) * mi / (sqrt(vi) / sbc2 + eps);
}

// ---------------------------------------------------------------------------
// GEMM form on the bfloat16 matrix cores (FP32 accumulation).  For one offset
// d the layer is a complex product
//   out[(o, s)][(x, a)] += sum_{(i, t)} W[o][i][d][s][t] (T_d(x) phi[i](x + d))[t][a]
// with M = 4 c_out, K = 4 c_in and N = 3 x the sites.  One workgroup takes 32
// sites (96 columns, six tiles of 16) and all output channels; per offset the
// 32 path products are formed once (FP64, then rounded), the weights of d and
// the transported inputs are staged in LDS as bfloat16 complex words, and
// each wave accumulates its output tiles with v_mfma_f32_16x16x16bf16_1k on
// the interleaved real embedding of the complex product (as the coarse apply:
// lane l holds A[l % 16][4 (l / 16) + i] and B[4 (l / 16) + i][l % 16]).
// Weights and inputs are rounded to bfloat16 once, before the launch.
constexpr int kPtcMaxCh = 24;                    // channels per layer on this path
constexpr int kPtcSites = 32;                    // sites per workgroup
constexpr int kPtcRows = 4 * kPtcMaxCh;          // complex rows (o, s) / K entries (i, t)
constexpr int kPtcCols = 3 * kPtcSites;          // complex columns (x, a)
constexpr int kPtcTiles = (kPtcRows / 8) * (kPtcCols / 16) / 4;   // output tiles per wave (of 4)

__device__ inline unsigned short bf16_of(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (unsigned short)((u >> 16) | 0x40u);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

__device__ inline unsigned bf16_word(double re, double im) {
  return (unsigned)bf16_of((float)re) | ((unsigned)bf16_of((float)im) << 16);
}

__device__ inline float bf16_lo(unsigned w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(unsigned w) { return __uint_as_float(w & 0xffff0000u); }

// weights as bfloat16 words [81][mrows][kcols], zero padded: row (o, s) and
// column (i, t) for the layer; for its adjoint (ADJ, the input gradient) row
// (i, t), column (o, s) and the entry conjugated (W^dag per spin block)
template <bool ADJ>
__global__ void k_ptc_weights_bf16(const c128 *__restrict__ W, int cin, int cout, int mrows, int kcols,
                                   unsigned *__restrict__ Wb) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)kPtcOffsets * mrows * kcols;
  if (e >= n) return;
  const int k = (int)(e / ((long long)mrows * kcols));
  const int rem = (int)(e - (long long)k * mrows * kcols);
  const int r = rem / kcols, c = rem - r * kcols;
  const int o = ADJ ? (c >> 2) : (r >> 2), s = ADJ ? (c & 3) : (r & 3);
  const int i = ADJ ? (r >> 2) : (c >> 2), t = ADJ ? (r & 3) : (c & 3);
  unsigned v = 0;
  if (o < cout && i < cin) {
    const c128 w = W[(((long long)o * cin + i) * kPtcOffsets + k) * 16 + 4 * s + t];
    v = bf16_word(w.re, ADJ ? -w.im : w.im);
  }
  Wb[e] = v;
}

// inputs as bfloat16 words, same layout [cin][12][V]
__global__ void k_fields_bf16(const c128 *__restrict__ x, long long n, unsigned *__restrict__ y) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) y[e] = bf16_word(x[e].re, x[e].im);
}

// T_d(x) in FP32 (the links rounded once): the path of path_transport
__device__ inline int path_transport_f(const Geom &g, const c128 *__restrict__ U, int x, const int d[4], c64 T[9]) {
  const long long V = g.V;
#pragma unroll
  for (int e = 0; e < 9; ++e) T[e] = c64{(e % 4 == 0) ? 1.f : 0.f, 0.f};
  int pos = x;
  for (int mu = 0; mu < 4; ++mu) {
    if (d[mu] == 0) continue;
    const SiteCoord c = decode(g, pos);
    float sg;
    bool in;
    const int nxt = neighbour(g, pos, c, mu, d[mu] > 0, &sg, &in);
    const int ls = d[mu] > 0 ? pos : nxt;
    c64 L[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) {
      // U_mu(pos) for a forward step, U_mu(pos - mu)^dag for a backward one
      const int src = d[mu] > 0 ? e : 3 * (e % 3) + e / 3;
      const c128 m = U[(long long)(mu * 9 + src) * V + ls];
      L[e] = c64{sg * (float)m.re, sg * (d[mu] > 0 ? (float)m.im : -(float)m.im)};
    }
    c64 P[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) P[3 * a + b] = T[3 * a] * L[b] + T[3 * a + 1] * L[3 + b] + T[3 * a + 2] * L[6 + b];
#pragma unroll
    for (int e = 0; e < 9; ++e) T[e] = P[e];
    pos = nxt;
  }
  return pos;
}

typedef short v4s_ptc __attribute__((ext_vector_type(4)));
typedef float v4f_ptc __attribute__((ext_vector_type(4)));

// ADJ: the input gradient, g_in[i](y) = sum_o sum_d W[o][i][d]^dag T_d(y - d)^dag g[o](y - d):
// rows (i, t), K (o, s), the transported field T_d(y - d)^dag g[o](y - d).
// cin here is the channel count of the field read (K), cout that of the output (rows).
template <bool ADJ>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_ptc_forward_bf16(Geom g, const c128 *__restrict__ U, int cin, int cout,
                                                          int mrows, int kcols, const unsigned *__restrict__ phib,
                                                          const unsigned *__restrict__ Wb, c128 *__restrict__ out) {
  __shared__ unsigned As[kPtcRows * (kPtcRows + 1)];
  __shared__ unsigned Bs[kPtcRows * (kPtcCols + 1)];
  __shared__ float Ts[kPtcSites][18];
  __shared__ int Ps[kPtcSites];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int x0 = blockIdx.x * kPtcSites;
  const long long V = g.V;
  const int lda = kPtcRows + 1, ldb = kPtcCols + 1;
  const int nt = kPtcCols / 16, ntiles = (mrows / 8) * nt;
  const int kq = lane >> 4, ri = lane & 1;
  v4f_ptc acc[kPtcTiles];
#pragma unroll
  for (int q = 0; q < kPtcTiles; ++q) acc[q] = v4f_ptc{0.f, 0.f, 0.f, 0.f};
  for (int k = 0; k < kPtcOffsets; ++k) {
    __syncthreads();                           // the previous offset's products are done with As, Bs
    if (t < kPtcSites) {
      int d[4];
      offset_of(k, d);
      const int x = x0 + t;
      c64 T[9];
      int pos = 0;
      if (x < g.V) {
        if (ADJ) {
          pos = back_offset(g, x, d);                    // the path from x - d ends at x
          (void)path_transport_f(g, U, pos, d, T);
        } else {
          pos = path_transport_f(g, U, x, d, T);
        }
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) T[e] = c64{0.f, 0.f};
      }
#pragma unroll
      for (int e = 0; e < 9; ++e) { Ts[t][2 * e] = T[e].re; Ts[t][2 * e + 1] = T[e].im; }
      Ps[t] = pos;
    }
    const unsigned *wk = Wb + (long long)k * mrows * kcols;
    for (int e = t; e < mrows * kcols; e += blockDim.x) {
      const int r = e / kcols, c = e - r * kcols;
      As[r * lda + c] = wk[e];
    }
    __syncthreads();
    // transported inputs of (site, channel) pairs: Bs[(i, t)][(x, a)]
    for (int e = t; e < kPtcSites * (kcols >> 2); e += blockDim.x) {
      const int xs = e % kPtcSites, i = e / kPtcSites;
      float qr[12], qi[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) { qr[c] = 0.f; qi[c] = 0.f; }
      if (i < cin && x0 + xs < g.V) {
        const unsigned *p = phib + (long long)i * 12 * V + Ps[xs];
        float pr[12], pi[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const unsigned wv = p[(long long)c * V];
          pr[c] = bf16_lo(wv);
          pi[c] = bf16_hi(wv);
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              // T[a][b] for the layer, conj(T[b][a]) for its adjoint
              const int te = ADJ ? 3 * b + a : 3 * a + b;
              const float tr = Ts[xs][2 * te], ti = ADJ ? -Ts[xs][2 * te + 1] : Ts[xs][2 * te + 1];
              re += tr * pr[3 * sp + b] - ti * pi[3 * sp + b];
              im += tr * pi[3 * sp + b] + ti * pr[3 * sp + b];
            }
            qr[3 * sp + a] = re;
            qi[3 * sp + a] = im;
          }
      }
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a)
          Bs[(4 * i + sp) * ldb + 3 * xs + a] = bf16_word(qr[3 * sp + a], qi[3 * sp + a]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPtcTiles; ++q) {
      const int tile = w + 4 * q;
      if (tile < ntiles) {                     // uniform per wave
        const int rt = tile / nt, ct = tile - rt * nt;
        const int crow = 8 * rt + ((lane & 15) >> 1), col = 16 * ct + (lane & 15);
        for (int st = 0; st < (kcols >> 3); ++st) {
          const int cj = 8 * st + 2 * kq;
          const unsigned m0 = As[crow * lda + cj], m1 = As[crow * lda + cj + 1];
          // Re row: (Mr, -Mi); Im row: (Mi, Mr)
          const unsigned a0 = ri ? ((m0 >> 16) | (m0 << 16)) : (m0 ^ 0x80000000u);
          const unsigned a1 = ri ? ((m1 >> 16) | (m1 << 16)) : (m1 ^ 0x80000000u);
          const unsigned b0 = Bs[cj * ldb + col], b1 = Bs[(cj + 1) * ldb + col];
          v4s_ptc av, bv;
          av[0] = (short)(a0 & 0xffffu); av[1] = (short)(a0 >> 16); av[2] = (short)(a1 & 0xffffu); av[3] = (short)(a1 >> 16);
          bv[0] = (short)(b0 & 0xffffu); bv[1] = (short)(b0 >> 16); bv[2] = (short)(b1 & 0xffffu); bv[3] = (short)(b1 >> 16);
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
  }
  // acc[q][r] = D[4 kq + r][col]: complex row 8 rt + 2 kq + (r >> 1), Re/Im = r & 1
#pragma unroll
  for (int q = 0; q < kPtcTiles; ++q) {
    const int tile = w + 4 * q;
    if (tile < ntiles) {
      const int rt = tile / nt, ct = tile - rt * nt;
      const int col = 16 * ct + (lane & 15);
      const int xs = col / 3, a = col - 3 * xs, x = x0 + xs;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int crow = 8 * rt + 2 * kq + h, o = crow >> 2, sp = crow & 3;
        if (o < cout && x < g.V) out[((long long)o * 12 + 3 * sp + a) * V + x] = c128{acc[q][2 * h], acc[q][2 * h + 1]};
      }
    }
  }
}

// The weight gradient on the bfloat16 matrix cores, per offset d a complex product
//   gW[o][i][d][s][t] = sum_x sum_a g[o](x)[s][a] conj((T_d(x) phi[i](x + d))[t][a])
// with M = 4 c_out rows (o, s), N = 4 c_in columns (i, t) and K = 3 V (site, colour).
// Workgroup (chunk, d) runs over its chunk of sites 32 at a time (K = 96 per step:
// the output gradients and the conjugated transported inputs staged in LDS) and
// writes its FP32 sums; k_ptc_gw_sum adds the chunks in a fixed order.
constexpr int kPtcGwCols = 4 * kPtcMaxCh;        // complex columns (i, t)

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
k_ptc_grad_weight_bf16(Geom g, const c128 *__restrict__ U, int cin, int cout, int mrows, int ncols, int chunk,
                       const unsigned *__restrict__ phib, const unsigned *__restrict__ gb, float2 *__restrict__ part) {
  __shared__ unsigned As[kPtcRows * (kPtcCols + 1)];
  __shared__ unsigned Bs[kPtcCols * (kPtcGwCols + 1)];
  __shared__ float Ts[kPtcSites][18];
  __shared__ int Ps[kPtcSites];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int k = blockIdx.y, ch = blockIdx.x;
  const int lo = ch * chunk, hi = min(lo + chunk, g.V);
  const long long V = g.V;
  const int lda = kPtcCols + 1, ldb = kPtcGwCols + 1;
  const int nt = ncols / 16, ntiles = (mrows / 8) * nt;
  const int kq = lane >> 4, ri = lane & 1;
  int d[4];
  offset_of(k, d);
  v4f_ptc acc[kPtcTiles];
#pragma unroll
  for (int q = 0; q < kPtcTiles; ++q) acc[q] = v4f_ptc{0.f, 0.f, 0.f, 0.f};
  for (int x0 = lo; x0 < hi; x0 += kPtcSites) {
    __syncthreads();                           // the previous step's products are done with As, Bs
    if (t < kPtcSites) {
      const int x = x0 + t;
      c64 T[9];
      int pos = 0;
      if (x < hi) {
        pos = path_transport_f(g, U, x, d, T);
      } else {
#pragma unroll
        for (int e = 0; e < 9; ++e) T[e] = c64{0.f, 0.f};
      }
#pragma unroll
      for (int e = 0; e < 9; ++e) { Ts[t][2 * e] = T[e].re; Ts[t][2 * e + 1] = T[e].im; }
      Ps[t] = pos;
    }
    // output gradients: As[(o, s)][(x, a)]
    for (int e = t; e < kPtcSites * (mrows >> 2); e += blockDim.x) {
      const int xs = e % kPtcSites, o = e / kPtcSites, x = x0 + xs;
      const bool live = o < cout && x < hi;
      const unsigned *p = gb + (long long)o * 12 * V + x;
#pragma unroll
      for (int c = 0; c < 12; ++c) As[(4 * o + c / 3) * lda + 3 * xs + c % 3] = live ? p[(long long)c * V] : 0u;
    }
    __syncthreads();
    // conjugated transported inputs: Bs[(x, a)][(i, t)]
    for (int e = t; e < kPtcSites * (ncols >> 2); e += blockDim.x) {
      const int xs = e % kPtcSites, i = e / kPtcSites;
      float qr[12], qi[12];
#pragma unroll
      for (int c = 0; c < 12; ++c) { qr[c] = 0.f; qi[c] = 0.f; }
      if (i < cin && x0 + xs < hi) {
        const unsigned *p = phib + (long long)i * 12 * V + Ps[xs];
        float pr[12], pi[12];
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          const unsigned wv = p[(long long)c * V];
          pr[c] = bf16_lo(wv);
          pi[c] = bf16_hi(wv);
        }
#pragma unroll
        for (int sp = 0; sp < 4; ++sp)
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int b = 0; b < 3; ++b) {
              const float tr = Ts[xs][2 * (3 * a + b)], ti = Ts[xs][2 * (3 * a + b) + 1];
              re += tr * pr[3 * sp + b] - ti * pi[3 * sp + b];
              im += tr * pi[3 * sp + b] + ti * pr[3 * sp + b];
            }
            qr[3 * sp + a] = re;
            qi[3 * sp + a] = -im;
          }
      }
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int a = 0; a < 3; ++a) Bs[(3 * xs + a) * ldb + 4 * i + sp] = bf16_word(qr[3 * sp + a], qi[3 * sp + a]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPtcTiles; ++q) {
      const int tile = w + 4 * q;
      if (tile < ntiles) {                     // uniform per wave
        const int rt = tile / nt, ct = tile - rt * nt;
        const int crow = 8 * rt + ((lane & 15) >> 1), col = 16 * ct + (lane & 15);
#pragma unroll 4
        for (int st = 0; st < kPtcCols / 8; ++st) {
          const int cj = 8 * st + 2 * kq;
          const unsigned m0 = As[crow * lda + cj], m1 = As[crow * lda + cj + 1];
          // Re row: (Mr, -Mi); Im row: (Mi, Mr)
          const unsigned a0 = ri ? ((m0 >> 16) | (m0 << 16)) : (m0 ^ 0x80000000u);
          const unsigned a1 = ri ? ((m1 >> 16) | (m1 << 16)) : (m1 ^ 0x80000000u);
          const unsigned b0 = Bs[cj * ldb + col], b1 = Bs[(cj + 1) * ldb + col];
          v4s_ptc av, bv;
          av[0] = (short)(a0 & 0xffffu); av[1] = (short)(a0 >> 16); av[2] = (short)(a1 & 0xffffu); av[3] = (short)(a1 >> 16);
          bv[0] = (short)(b0 & 0xffffu); bv[1] = (short)(b0 >> 16); bv[2] = (short)(b1 & 0xffffu); bv[3] = (short)(b1 >> 16);
          acc[q] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc[q], 0, 0, 0);
        }
      }
    }
  }
  // acc[q][r] = D[4 kq + r][col]: complex row 8 rt + 2 kq + (r >> 1), Re/Im = r & 1
  const long long nW = (long long)cout * cin * kPtcOffsets * 16;
#pragma unroll
  for (int q = 0; q < kPtcTiles; ++q) {
    const int tile = w + 4 * q;
    if (tile < ntiles) {
      const int rt = tile / nt, ct = tile - rt * nt;
      const int col = 16 * ct + (lane & 15), i = col >> 2, tc = col & 3;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int crow = 8 * rt + 2 * kq + h, o = crow >> 2, sp = crow & 3;
        if (o < cout && i < cin)
          part[ch * nW + (((long long)o * cin + i) * kPtcOffsets + k) * 16 + 4 * sp + tc] =
              float2{acc[q][2 * h], acc[q][2 * h + 1]};
      }
    }
  }
}

// gW[e] = sum over the chunks of part[chunk][e], in chunk order, in FP64
__global__ void k_ptc_gw_sum(long long nW, int nchunk, const float2 *__restrict__ part, c128 *__restrict__ gW) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nW) return;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    const float2 v = part[c * nW + e];
    re += v.x;
    im += v.y;
  }
  gW[e] = c128{re, im};
}

}  // namespace

void launch_adam(long long n, double *p, const double *g, double *m, double *v, double lr, double b1, double b2,
                 double eps, int t, hipStream_t st) {
  if (n <= 0) return;
  const double bc1 = 1.0 - pow(b1, (double)t), sbc2 = sqrt(1.0 - pow(b2, (double)t));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, 256)), dim3(256), 0, st, n, p, g, m, v, lr, b1, b2, eps, bc1, sbc2);
  LQ_HIP(hipGetLastError());
}

void launch_proj_loss(const int L[4], const int agg[4], int nout, const c128 *X, int K, const c128 *u, double *part,
                      double *loss, c128 *gX, int *status, hipStream_t st) {
  ProjGeom pg;
  pg.bvol = 1;
  pg.V = 1;
  int nblk = 1;
  for (int m = 0; m < 4; ++m) {
    pg.L[m] = L[m];
    pg.agg[m] = agg[m];
    pg.bvol *= agg[m];
    pg.V *= L[m];
    nblk *= L[m] / agg[m];
  }
  hipLaunchKernelGGL(k_proj_loss, dim3(2 * nblk), dim3(256), 0, st, pg, nout, X, K, u, part, gX, status);
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_rows, dim3(1), dim3(256), 0, st, 2 * nblk, part, loss);
  LQ_HIP(hipGetLastError());
}

void launch_mod_relu_backward(int V, int channels, const c128 *phi, const double *b, const c128 *gout, c128 *gphi,
                              double *gb, double *scratch, hipStream_t st) {
  hipLaunchKernelGGL(k_mod_relu_grad, dim3(blocks_for(V, 256), channels), dim3(256), 0, st, V, phi, b, gout, gphi,
                     scratch);
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_sum_rows, dim3(channels), dim3(256), 0, st, V, scratch, gb);
  LQ_HIP(hipGetLastError());
}

void launch_mod_relu(int V, int channels, const c128 *phi, const double *b, c128 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_mod_relu, dim3(blocks_for(V, 256), channels), dim3(256), 0, st, V, phi, b, out);
  LQ_HIP(hipGetLastError());
}

void launch_ptc_backward(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                         const c128 *gout, c128 *gin, c128 *gW, hipStream_t st) {
  if (gin) {
    hipLaunchKernelGGL(k_ptc_grad_input, dim3(blocks_for(g.V, 256), cin), dim3(256), 0, st, g, U, cout, gout, cin, W,
                       gin);
    LQ_HIP(hipGetLastError());
  }
  if (gW) {
    hipLaunchKernelGGL(k_ptc_grad_weight, dim3(cout * cin * kPtcOffsets), dim3(256), 0, st, g, U, cin, phi, cout,
                       gout, gW);
    LQ_HIP(hipGetLastError());
  }
}

void launch_ptc_forward(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W, c128 *out,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_ptc_forward, dim3(blocks_for(g.V, 256), cout), dim3(256), 0, st, g, U, cin, phi, W, out);
  LQ_HIP(hipGetLastError());
}

size_t ptc_bf16_scratch_words(int V, int cin, int cout) {
  const int mrows = ((cout + 1) / 2) * 8, kcols = ((cin + 1) / 2) * 8;
  return (size_t)kPtcOffsets * mrows * kcols + (size_t)cin * 12 * V;
}

void launch_ptc_forward_bf16(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                             c128 *out, unsigned *scratch, hipStream_t st) {
  const int mrows = ((cout + 1) / 2) * 8, kcols = ((cin + 1) / 2) * 8;
  unsigned *Wb = scratch, *phib = scratch + (size_t)kPtcOffsets * mrows * kcols;
  const long long nw = (long long)kPtcOffsets * mrows * kcols, nf = (long long)cin * 12 * g.V;
  hipLaunchKernelGGL((k_ptc_weights_bf16<false>), dim3(blocks_for(nw, 256)), dim3(256), 0, st, W, cin, cout, mrows,
                     kcols, Wb);
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_fields_bf16, dim3(blocks_for(nf, 256)), dim3(256), 0, st, phi, nf, phib);
  LQ_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_ptc_forward_bf16<false>), dim3(blocks_for(g.V, kPtcSites)), dim3(256), 0, st, g, U, cin, cout,
                     mrows, kcols, phib, Wb, out);
  LQ_HIP(hipGetLastError());
}

namespace {
struct PtcBwdPlan {
  int mrows_in, kcols_in;                        // the adjoint product (input gradient)
  int mrows_w, ncols_w, chunk, nchunk;           // the weight-gradient product
  size_t off_phi, off_w, off_part, words;
};

PtcBwdPlan ptc_bwd_plan(int V, int cin, int cout) {
  PtcBwdPlan p;
  p.mrows_in = ((cin + 1) / 2) * 8;
  p.kcols_in = ((cout + 1) / 2) * 8;
  p.mrows_w = ((cout + 1) / 2) * 8;
  p.ncols_w = ((cin + 3) / 4) * 16;
  // chunks of about 2048 sites (at most 32), a multiple of the 32 sites of a step
  const int want = std::max(1, std::min(32, (V + 2047) / 2048));
  p.chunk = ((V + want - 1) / want + kPtcSites - 1) / kPtcSites * kPtcSites;
  p.nchunk = (V + p.chunk - 1) / p.chunk;
  const size_t nW = (size_t)cout * cin * kPtcOffsets * 16;
  p.off_phi = (size_t)cout * 12 * V;
  p.off_w = p.off_phi + (size_t)cin * 12 * V;
  p.off_part = p.off_w + (size_t)kPtcOffsets * p.mrows_in * p.kcols_in;
  p.off_part = (p.off_part + 1) & ~(size_t)1;     // float2 alignment
  p.words = p.off_part + 2 * (size_t)p.nchunk * nW;
  return p;
}
}  // namespace

size_t ptc_bf16_backward_scratch_words(int V, int cin, int cout) { return ptc_bwd_plan(V, cin, cout).words; }

void launch_ptc_backward_bf16(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                              const c128 *gout, c128 *gin, c128 *gW, unsigned *scratch, hipStream_t st) {
  const PtcBwdPlan p = ptc_bwd_plan(g.V, cin, cout);
  unsigned *gb = scratch, *phib = scratch + p.off_phi, *Wb = scratch + p.off_w;
  float2 *part = reinterpret_cast<float2 *>(scratch + p.off_part);
  const long long ng = (long long)cout * 12 * g.V;
  hipLaunchKernelGGL(k_fields_bf16, dim3(blocks_for(ng, 256)), dim3(256), 0, st, gout, ng, gb);
  LQ_HIP(hipGetLastError());
  if (gin) {
    // the adjoint product: rows (i, t) of the input channels, K (o, s) of the output channels
    const long long nw = (long long)kPtcOffsets * p.mrows_in * p.kcols_in;
    hipLaunchKernelGGL((k_ptc_weights_bf16<true>), dim3(blocks_for(nw, 256)), dim3(256), 0, st, W, cin, cout,
                       p.mrows_in, p.kcols_in, Wb);
    LQ_HIP(hipGetLastError());
    hipLaunchKernelGGL((k_ptc_forward_bf16<true>), dim3(blocks_for(g.V, kPtcSites)), dim3(256), 0, st, g, U, cout,
                       cin, p.mrows_in, p.kcols_in, gb, Wb, gin);
    LQ_HIP(hipGetLastError());
  }
  if (gW) {
    const long long nf = (long long)cin * 12 * g.V, nW = (long long)cout * cin * kPtcOffsets * 16;
    hipLaunchKernelGGL(k_fields_bf16, dim3(blocks_for(nf, 256)), dim3(256), 0, st, phi, nf, phib);
    LQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ptc_grad_weight_bf16, dim3(p.nchunk, kPtcOffsets), dim3(256), 0, st, g, U, cin, cout,
                       p.mrows_w, p.ncols_w, p.chunk, phib, gb, part);
    LQ_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ptc_gw_sum, dim3(blocks_for(nW, 256)), dim3(256), 0, st, nW, p.nchunk, part, gW);
    LQ_HIP(hipGetLastError());
  }
}

}  // namespace lq
