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

}  // namespace lq
