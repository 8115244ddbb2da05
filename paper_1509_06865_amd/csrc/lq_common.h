// Internal definitions shared by the HIP translation units of liblqmg.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace lq {

// ---------------------------------------------------------------- complex ---
template <typename T> struct cplx { T re, im; };
using c64 = cplx<float>;
using c128 = cplx<double>;

template <typename T> __host__ __device__ inline cplx<T> mk(T r, T i) { return {r, i}; }
template <typename T> __host__ __device__ inline cplx<T> operator+(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator-(cplx<T> a) { return {-a.re, -a.im}; }
template <typename T> __host__ __device__ inline cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> __host__ __device__ inline cplx<T> operator*(T s, cplx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> __host__ __device__ inline cplx<T> conj(cplx<T> a) { return {a.re, -a.im}; }
// conj(a) * b
template <typename T> __host__ __device__ inline cplx<T> cmul_conj(cplx<T> a, cplx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
// i * a and -i * a
template <typename T> __host__ __device__ inline cplx<T> times_i(cplx<T> a) { return {-a.im, a.re}; }
template <typename T> __host__ __device__ inline cplx<T> times_mi(cplx<T> a) { return {a.im, -a.re}; }
template <typename T> __host__ __device__ inline T norm2(cplx<T> a) { return a.re * a.re + a.im * a.im; }
template <typename To, typename From> __host__ __device__ inline cplx<To> cast(cplx<From> a) {
  return {(To)a.re, (To)a.im};
}

// --------------------------------------------------------------- geometry ---
// Lattice sites are stored blocked: the lattice is cut into blocks of extent
// b[mu]; site s = A * bvol + l with A the block index (A_x fastest) and l the
// site inside the block (l_x fastest).  One block covering the whole lattice
// is the canonical ordering n = x + X*(y + Y*(z + Z*t)).
struct Geom {
  int L[4];       // lattice extents
  int b[4];       // block extents
  int nb[4];      // blocks per direction
  int sl[4];      // strides of the local coordinate (prod of b below mu)
  int sA[4];      // strides of the block coordinate (prod of nb below mu)
  int bvol;       // sites per block
  int nblk;       // number of blocks
  int V;          // sites
  int tbc;        // -1 antiperiodic, +1 periodic in t
};

inline Geom make_geom(const int L[4], const int b[4], int tbc) {
  Geom g;
  int sl = 1, sA = 1;
  for (int m = 0; m < 4; ++m) {
    g.L[m] = L[m]; g.b[m] = b[m]; g.nb[m] = L[m] / b[m];
    g.sl[m] = sl; g.sA[m] = sA; sl *= b[m]; sA *= g.nb[m];
  }
  g.bvol = sl; g.nblk = sA; g.V = sl * sA; g.tbc = tbc;
  return g;
}

// Decoded site: local and block coordinates.
struct SiteCoord { int l[4]; int a[4]; int blk; int loc; };

__host__ __device__ inline SiteCoord decode(const Geom &g, int s) {
  SiteCoord c;
  c.blk = s / g.bvol;
  c.loc = s - c.blk * g.bvol;
  int r = c.loc;
  for (int m = 0; m < 3; ++m) { int q = r / g.b[m]; c.l[m] = r - q * g.b[m]; r = q; }
  c.l[3] = r;
  r = c.blk;
  for (int m = 0; m < 3; ++m) { int q = r / g.nb[m]; c.a[m] = r - q * g.nb[m]; r = q; }
  c.a[3] = r;
  return c;
}

// Neighbour of site s (coordinates c) in direction mu, forward (+1) or
// backward; *sign receives the boundary sign of that hop; *inside tells
// whether the neighbour lies in the same block without wrapping.
__host__ __device__ inline int neighbour(const Geom &g, int s, const SiteCoord &c, int mu,
                                         bool fwd, float *sign, bool *inside) {
  int bm = g.b[mu];
  *sign = 1.f;
  if (fwd) {
    if (c.l[mu] + 1 < bm) { *inside = true; return s + g.sl[mu]; }
    *inside = false;
    int t = s - (bm - 1) * g.sl[mu];
    if (c.a[mu] + 1 < g.nb[mu]) t += g.sA[mu] * g.bvol;
    else { t -= (g.nb[mu] - 1) * g.sA[mu] * g.bvol; if (mu == 3) *sign = (float)g.tbc; }
    return t;
  } else {
    if (c.l[mu] > 0) { *inside = true; return s - g.sl[mu]; }
    *inside = false;
    int t = s + (bm - 1) * g.sl[mu];
    if (c.a[mu] > 0) t -= g.sA[mu] * g.bvol;
    else { t += (g.nb[mu] - 1) * g.sA[mu] * g.bvol; if (mu == 3) *sign = (float)g.tbc; }
    return t;
  }
}

// ---------------------------------------------------------------- launch ----
#define LQ_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) throw ::lq::HipError(e_, #call, __FILE__, __LINE__); \
  } while (0)

struct HipError {
  hipError_t err; const char *what; const char *file; int line;
  HipError(hipError_t e, const char *w, const char *f, int l) : err(e), what(w), file(f), line(l) {}
};

inline unsigned blocks_for(long long n, int threads) { return (unsigned)((n + threads - 1) / threads); }

// The dispatcher hands consecutive workgroups of a launch to the 8 XCDs in
// turn, and each XCD has its own L2.  Renumbering the workgroups so that XCD x
// runs one contiguous range of tiles keeps stencil neighbours in one L2.  A
// bijection of [0, n) for any n.
constexpr int kNumXcd = 8;
__device__ inline int xcd_tile(int b, int n) {
  const int q = n / kNumXcd, r = n % kNumXcd;
  const int x = b % kNumXcd, k = b / kNumXcd;
  return x * q + (x < r ? x : r) + k;
}

// Per-rhs scalar passed to kernels: shifts, coefficients.
constexpr int kMaxRhs = 16;

// Rows of a stored clover field [kCloverRows][V] (42 used; a multiple of 12,
// so the layout changes of [n][12][V] fields apply to it).
constexpr int kCloverRows = 48;

}  // namespace lq
