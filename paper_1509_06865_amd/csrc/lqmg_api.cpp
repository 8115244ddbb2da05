// Host side of liblqmg: the context, batched (flexible) GMRES, the multigrid
// cycle and setup, Rayleigh quotient iteration (Alg. 1) and the C ABI.
// Every numerical step runs in the HIP kernels of this library; the host only
// keeps the small Hessenberg / Givens state of the Krylov solvers, the
// eigenvalue bookkeeping of Alg. 1 and the control flow.
#include "lqmg.h"
#include "lq_kernels.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

using namespace lq;
using cd = std::complex<double>;

namespace {

struct ApiError {
  int code;
  std::string msg;
};

[[noreturn]] void fail(int code, const std::string &m) { throw ApiError{code, m}; }

template <typename T> struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  T *get(size_t count) {
    if (count <= n && p) return p;
    release();
    if (count == 0) count = 1;
    if (hipMalloc(&p, count * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      p = nullptr;
      size_t fr = 0, tot = 0;
      (void)hipMemGetInfo(&fr, &tot);
      fail(LQ_ERR_OOM, "device allocation of " + std::to_string(count * sizeof(T)) + " bytes failed (" +
                           std::to_string(fr >> 20) + " MiB free of " + std::to_string(tot >> 20) + ")");
    }
    // new buffers start zeroed (reduction counters rely on it)
    if (hipMemset(p, 0, count * sizeof(T)) != hipSuccess) fail(LQ_ERR_HIP, "hipMemset failed");
    n = count;
    return p;
  }
};

double now() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// Progress lines on stderr when LQMG_VERBOSE is set (long calls stay observable).
bool verbose() {
  static const bool v = std::getenv("LQMG_VERBOSE") != nullptr;
  return v;
}

template <typename T> struct MGData {
  DevBuf<cplx<T>> U;    // blocked links (T precision)
  DevBuf<cplx<T>> C;    // blocked clover term (T precision), when c_sw != 0
  DevBuf<cplx<T>> P;    // [Nv][12][V]
  DevBuf<cplx<T>> Qc;   // [nA][5][n2][n2]
  DevBuf<cplx<T>> P2;   // third level: [Nv2][nA][n2]
  DevBuf<cplx<T>> Qc2;  // [nA2][5][n22][n22]
};

// Device-side state of one batched GMRES: Hessenberg columns, Givens
// rotations, per-system activity and the reduction outputs.
struct KState {
  DevBuf<c128> bH, bsn, bg, bh1, bh2, bnrm, bcoef, bY;
  DevBuf<double> bcs, bbn;
  DevBuf<int> bact, bkk, bbad;
  c128 *H, *sn, *g, *h1, *h2, *nrm2, *coef, *Y;
  double *cs, *bn;
  int *active, *kk, *bad;
  void alloc(int m, int nrhs) {
    H = bH.get((size_t)nrhs * (m + 1) * m);
    sn = bsn.get((size_t)nrhs * m);
    g = bg.get((size_t)nrhs * (m + 1));
    h1 = bh1.get((size_t)(m + 1) * nrhs);
    h2 = bh2.get((size_t)(m + 1) * nrhs);
    nrm2 = bnrm.get(nrhs);
    coef = bcoef.get(nrhs);
    Y = bY.get((size_t)m * nrhs);
    cs = bcs.get((size_t)nrhs * m);
    bn = bbn.get(nrhs);
    active = bact.get(nrhs);
    kk = bkk.get(nrhs);
    bad = bbad.get(1);
  }
};

// Work vectors of one batched Krylov solve.
template <typename T> struct KrylovWork {
  DevBuf<cplx<T>> V, Z, r;
  DevBuf<c128> scratch;
  KState st;
};

}  // namespace

struct lq_ctx {
  int L[4];
  int tbc;
  hipStream_t st;
  std::string err;
  Geom gcan;
  int dev;

  bool have = false;
  lq_mg_params p;
  double m0 = 0;
  int Nv = 0;
  int agg[4];
  Geom g;
  CoarseGeom cg;
  DevBuf<c128> U64;                 // blocked FP64 links (outer operator)
  double csw = 0;                   // clover coefficient (lq_clover); 0: plain Wilson
  DevBuf<c128> clov_can, clov64;    // clover term: canonical (from lq_clover), blocked (mg_setup)
  DevBuf<c64> clov_can32;           // canonical FP32 copy (q_apply_c64)
  MGData<double> d64;
  MGData<float> d32;
  DevBuf<c128> W;                   // test vectors, blocked, FP64
  DevBuf<c128> P64;                 // P in FP64 (source of the FP32 copy)
  DevBuf<int> blocks[2];
  int nblocks[2] = {0, 0};
  DevBuf<int> status;
  DevBuf<c128> red_scratch, red_out, coef, gram_scratch;
  DevBuf<int> ints;                 // small per-call integer arrays
  // workspaces
  KrylovWork<double> fine_kw;
  KrylovWork<double> coarse_kw64;
  KrylovWork<float> coarse_kw32;
  DevBuf<c128> tmpA, tmpB;          // FP64 fine work
  DevBuf<c64> f32a, f32b, f32c;     // FP32 fine work (mixed cycle)
  DevBuf<c128> f64a, f64b;          // FP64 fine work (cycle)
  DevBuf<c128> c64a, c64b;          // coarse work (FP64)
  DevBuf<c64> c32a, c32b;           // coarse work (FP32)
  DevBuf<c128> parts64, pc64;
  DevBuf<c64> parts32, pc32;
  DevBuf<c128> eig;                 // RQI vectors, blocked FP64 [n][12][V]
  DevBuf<const c128 *> src_cols;    // addresses of the fields P is built from (device)
  DevBuf<c128> defl_tmp, defl_u, defl_r;   // Galerkin correction work           // Rayleigh-Ritz: gathered unconverged vectors
  DevBuf<c128> minus_one, plus_one; // constant coefficient arrays [kMaxRhs]
  DevBuf<double> coarse_sig;        // shifts of the current coarse solve [kMaxRhs]
  DevBuf<bf16c> QcB;                // the FP32 Q_c in bfloat16 (coarse_bf16)
  DevBuf<double> net_scratch;       // per-site partial sums of the network's bias gradients
  DevBuf<unsigned> ptc_bf16;        // bfloat16 weights and inputs of the matrix-core layer
  // third level (n_levels == 3): aggregates of the coarse lattice
  int n_levels = 2;
  int Nv2 = 0;
  int agg2[4] = {1, 1, 1, 1};
  Level2Geom l2g;
  CoarseGeom cg2;
  DevBuf<c128> P2_64, W2;            // level-2 interpolation (FP64) and the level-1 vectors it is built from
  KrylovWork<double> smooth1_kw64, coarse2_kw64;
  KrylovWork<float> smooth1_kw32, coarse2_kw32;
  DevBuf<c128> l1w64, l2w64;         // level-1 / level-2 work vectors (FP64)
  DevBuf<c64> l1w32, l2w32;          // (FP32)
  DevBuf<c128> parts2_64, pc2_64;
  DevBuf<c64> parts2_32, pc2_32;
  DevBuf<c128> lma_V, lma_W, lma_X;  // approximate low-mode averaging: kept vectors, work fields
  DevBuf<c128> lma_out;
  DevBuf<c128> lz_basis[2], lz_tmp;  // restarted Lanczos: the basis and its restarted copy, Q v
  int coarse_iters = 0;
  // captured coarse-GMRES chunks, keyed by shape, step range and every pointer
  // they use; cap_st is the private stream they are captured on
  std::map<std::vector<uint64_t>, hipGraphExec_t> graphs;
  hipStream_t cap_st = nullptr;
  ~lq_ctx() {
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
    if (cap_st) (void)hipStreamDestroy(cap_st);
  }
};

namespace {

// ---------------------------------------------------------------------------
// Device scratch of the allocation-free entry point (lq_inner_products_noalloc):
// a fixed array in the library's code object, one copy per device, held until
// the process ends.  Host code never uses its name as an address: each
// device's address is resolved once, with that device current, and kept.
// ---------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = (size_t)LQ_NOALLOC_SCRATCH_BYTES;
constexpr size_t kNoAllocOutBytes = 64 * 1024;          // [nb][nw] results, nb <= 192, nw <= 16
static_assert(192 * 16 * sizeof(c128) <= kNoAllocOutBytes, "result area too small");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Resolve the scratch array's address on device dev (current).  Returns false
// if the runtime cannot give it.
bool resolve_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return false;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[dev]) return true;
  void *p = nullptr;
  if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
    (void)hipGetLastError();
    return false;
  }
  g_scratch_ptr[dev] = p;
  return true;
}

void *scratch_on(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[dev];
}

void sync(lq_ctx *c) { LQ_HIP(hipStreamSynchronize(c->st)); }

uint64_t key_bits(const void *p) { return (uint64_t)(uintptr_t)p; }
uint64_t key_bits(double d) {
  uint64_t u;
  std::memcpy(&u, &d, sizeof(u));
  return u;
}

// Release every captured graph (after the stream has drained).
void drop_graphs(lq_ctx *c) {
  if (c->graphs.empty()) return;
  sync(c);
  for (auto &kv : c->graphs) LQ_HIP(hipGraphExecDestroy(kv.second));
  c->graphs.clear();
}

// The executable graph of `body` (launches on c->st only, no host waits, no
// memsets), captured on first use of `key` on a private stream and reused.
// The cache holds at most 256 graphs; when full it is emptied after the
// stream has drained.
hipGraphExec_t chunk_graph(lq_ctx *c, const std::vector<uint64_t> &key, const std::function<void()> &body) {
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) return it->second;
  if (c->graphs.size() >= 256) drop_graphs(c);
  if (!c->cap_st) LQ_HIP(hipStreamCreateWithFlags(&c->cap_st, hipStreamNonBlocking));
  const hipStream_t orig = c->st;
  LQ_HIP(hipStreamBeginCapture(c->cap_st, hipStreamCaptureModeRelaxed));
  c->st = c->cap_st;
  hipGraph_t g = nullptr;
  try {
    body();
  } catch (...) {
    c->st = orig;
    if (hipStreamEndCapture(c->cap_st, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
    throw;
  }
  c->st = orig;
  LQ_HIP(hipStreamEndCapture(c->cap_st, &g));
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  LQ_HIP(e);
  c->graphs.emplace(key, ex);
  return ex;
}

template <typename T> void zero(lq_ctx *c, cplx<T> *p, size_t n) {
  LQ_HIP(hipMemsetAsync(p, 0, n * sizeof(cplx<T>), c->st));
}
template <typename T> void copy(lq_ctx *c, cplx<T> *dst, const cplx<T> *src, size_t n) {
  LQ_HIP(hipMemcpyAsync(dst, src, n * sizeof(cplx<T>), hipMemcpyDeviceToDevice, c->st));
}

// Inner products <v_i,k, w_k>, returned to the host as [nv][nrhs].
template <typename T>
std::vector<cd> dots(lq_ctx *c, int nv, const cplx<T> *vbase, long long vstride, long long rstride,
                     const cplx<T> *w, long long wstride, long long n, int nrhs) {
  std::vector<cd> out((size_t)nv * nrhs);
  if (nv == 0) return out;
  c128 *sc = c->red_scratch.get(dots_scratch_elems(nv, nrhs));
  c128 *o = c->red_out.get((size_t)nv * nrhs);
  launch_dots<T>(nv, vbase, vstride, rstride, w, wstride, n, nrhs, o, sc, c->st);
  LQ_HIP(hipMemcpyAsync(out.data(), o, out.size() * sizeof(c128), hipMemcpyDeviceToHost, c->st));
  sync(c);
  return out;
}

// w_k += sign * sum_i h[i][k] v_i,k with h given on the host
template <typename T>
void axpys(lq_ctx *c, int nv, const cplx<T> *vbase, long long vstride, long long rstride,
           const std::vector<cd> &h, cplx<T> *w, long long wstride, long long n, int nrhs, double sign) {
  if (nv == 0) return;
  c128 *d = c->coef.get((size_t)nv * nrhs);
  LQ_HIP(hipMemcpyAsync(d, h.data(), (size_t)nv * nrhs * sizeof(c128), hipMemcpyHostToDevice, c->st));
  launch_multi_axpy<T>(nv, vbase, vstride, rstride, d, w, wstride, n, nrhs, sign, c->st);
  sync(c);   // the host vector h may be released after return
}

template <typename T>
void scale(lq_ctx *c, const std::vector<cd> &a, const cplx<T> *x, long long xs, cplx<T> *y, long long ys,
           long long n, int nrhs, bool acc) {
  c128 *d = c->coef.get((size_t)nrhs);
  LQ_HIP(hipMemcpyAsync(d, a.data(), (size_t)nrhs * sizeof(c128), hipMemcpyHostToDevice, c->st));
  launch_scale<T>(d, x, xs, y, ys, n, nrhs, acc, c->st);
  sync(c);
}

// <E_i, W_k> for a shared basis E (read once), returned as [nb][nw]
std::vector<cd> gram(lq_ctx *c, int nb, const c128 *E, long long estride, int nw, const c128 *W, long long wstride,
                     long long n) {
  std::vector<cd> out((size_t)nb * nw);
  if (nb == 0 || nw == 0) return out;
  c128 *sc = c->gram_scratch.get(gram_scratch_elems(n));
  c128 *o = c->red_out.get((size_t)nb * nw);
  launch_gram(nb, E, estride, nw, W, wstride, n, o, sc, c->st);
  LQ_HIP(hipMemcpyAsync(out.data(), o, out.size() * sizeof(c128), hipMemcpyDeviceToHost, c->st));
  sync(c);
  return out;
}

// U_k (+)= sign * sum_i Y[i][k] E_i, Y given on the host as [nb][nw]
void combine(lq_ctx *c, int nb, const c128 *E, long long estride, int nw, const std::vector<cd> &Y, double sign,
             c128 *U, long long ustride, long long n, bool accumulate) {
  if (nb == 0 || nw == 0) return;
  std::vector<cd> Ys(Y.size());
  for (size_t e = 0; e < Y.size(); ++e) Ys[e] = sign * Y[e];
  c128 *d = c->coef.get(Ys.size());
  LQ_HIP(hipMemcpyAsync(d, Ys.data(), Ys.size() * sizeof(c128), hipMemcpyHostToDevice, c->st));
  launch_combine(nb, E, estride, nw, d, U, ustride, n, accumulate, c->st);
  sync(c);
}

template <typename T>
std::vector<double> norms(lq_ctx *c, const cplx<T> *w, long long n, int nrhs) {
  std::vector<double> r(nrhs);
  for (int k0 = 0; k0 < nrhs; k0 += kMaxRhs) {           // one launch per 16 vectors
    const int nk = std::min(kMaxRhs, nrhs - k0);
    auto d = dots<T>(c, 1, w + k0 * n, 0, n, w + k0 * n, n, n, nk);
    for (int k = 0; k < nk; ++k) r[k0 + k] = std::sqrt(std::max(0.0, d[k].real()));
  }
  return r;
}

// ---------------------------------------------------------------------------
// Batched restarted (flexible) GMRES from x = 0.  nrhs independent systems
// share every kernel launch; each keeps its own Hessenberg matrix and stops on
// its own.  Orthogonalisation: classical Gram-Schmidt applied twice.
// ---------------------------------------------------------------------------
template <typename T> struct KOps {
  std::function<void(const cplx<T> *, cplx<T> *)> apply;                       // y = A x
  std::function<void(const cplx<T> *, cplx<T> *)> precond;                     // z = M v, may be empty
  std::function<void(const cplx<T> *, const cplx<T> *, cplx<T> *)> resid;      // r = b - A x
};

// Fixed-step form: exactly m Arnoldi steps from x = 0 (one cycle, no
// restart, no convergence test) with no value read back to the host, so the
// whole solve is one asynchronous stream of launches (a polynomial smoother
// or a fixed-accuracy inner solve).
template <typename T>
void gmres_fixed(lq_ctx *c, KrylovWork<T> &kw, long long n, int nrhs, const KOps<T> &ops, const cplx<T> *b,
                 cplx<T> *x, int m) {
  const bool flex = (bool)ops.precond;
  cplx<T> *Vb = kw.V.get((size_t)(m + 1) * nrhs * n);
  cplx<T> *Zb = flex ? kw.Z.get((size_t)m * nrhs * n) : nullptr;
  KState &S = kw.st;
  S.alloc(m, nrhs);
  const long long vs = (long long)nrhs * n;
  c128 *sc = kw.scratch.get(dots_scratch_elems(m + 1, nrhs));
  Shifts one;
  for (int k = 0; k < kMaxRhs; ++k) one.s[k] = 1.0;
  launch_set_shifts(one, nrhs, S.bn, c->st);            // tolerance 0: only bn > 0 matters
  launch_dots<T>(1, b, 0, n, b, n, n, nrhs, S.nrm2, sc, c->st);
  launch_arnoldi_start(nrhs, m, S.nrm2, S.bn, 0.0, S.g, S.active, S.kk, S.coef, c->st);
  launch_scale<T>(S.coef, b, n, Vb, n, n, nrhs, false, c->st);
  for (int j = 0; j < m; ++j) {
    cplx<T> *vj = Vb + j * vs, *w = Vb + (j + 1) * vs;
    const cplx<T> *src = vj;
    if (flex) {
      ops.precond(vj, Zb + j * vs);
      src = Zb + j * vs;
    }
    ops.apply(src, w);
    launch_dots<T>(j + 1, Vb, vs, n, w, n, n, nrhs, S.h1, sc, c->st, S.active);
    launch_multi_axpy<T>(j + 1, Vb, vs, n, S.h1, w, n, n, nrhs, -1.0, c->st, S.active);
    launch_dots<T>(j + 1, Vb, vs, n, w, n, n, nrhs, S.h2, sc, c->st, S.active);
    launch_multi_axpy<T>(j + 1, Vb, vs, n, S.h2, w, n, n, nrhs, -1.0, c->st, S.active);
    launch_dots<T>(1, w, 0, n, w, n, n, nrhs, S.nrm2, sc, c->st, S.active);
    launch_arnoldi_update(j, m, nrhs, S.h1, S.h2, S.nrm2, S.H, S.cs, S.sn, S.g, S.bn, 0.0, S.active, S.kk, S.coef,
                          S.bad, c->st);
    launch_scale<T>(S.coef, w, n, w, n, n, nrhs, false, c->st);
  }
  launch_arnoldi_solve(m, nrhs, S.H, S.g, S.kk, S.Y, c->st);
  launch_multi_axpy<T>(m, flex ? Zb : Vb, vs, n, S.Y, x, n, n, nrhs, 1.0, c->st);
}

template <typename T>
bool gmres_batched(lq_ctx *c, KrylovWork<T> &kw, long long n, int nrhs, const KOps<T> &ops, const cplx<T> *b,
                   cplx<T> *x, int m, int max_restarts, double tol, int *iters, double *relres,
                   int check_every, const std::vector<uint64_t> *graph_id = nullptr) {
  // All Arnoldi bookkeeping stays on the device; the host waits only once per
  // restart cycle, and in between every check_every steps to stop early.
  // With graph_id (the identity of ops: every pointer and value their launches
  // use) the steps between two checks are replayed as one captured graph.
  const bool flex = (bool)ops.precond;
  cplx<T> *Vb = kw.V.get((size_t)(m + 1) * nrhs * n);
  cplx<T> *Zb = flex ? kw.Z.get((size_t)m * nrhs * n) : nullptr;
  cplx<T> *r = kw.r.get((size_t)nrhs * n);
  KState &S = kw.st;
  S.alloc(m, nrhs);
  LQ_HIP(hipMemsetAsync(S.bad, 0, sizeof(int), c->st));
  const long long vs = (long long)nrhs * n;     // stride between basis vectors
  c128 *sc = kw.scratch.get(dots_scratch_elems(m + 1, nrhs));
  // ||b_k||
  launch_dots<T>(1, b, 0, n, b, n, n, nrhs, S.nrm2, sc, c->st);
  std::vector<c128> h_nrm(nrhs);
  LQ_HIP(hipMemcpyAsync(h_nrm.data(), S.nrm2, nrhs * sizeof(c128), hipMemcpyDeviceToHost, c->st));
  sync(c);
  std::vector<double> bn(nrhs), beta(nrhs);
  for (int k = 0; k < nrhs; ++k) bn[k] = beta[k] = std::sqrt(std::max(0.0, h_nrm[k].re));
  LQ_HIP(hipMemcpyAsync(S.bn, bn.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, c->st));
  zero<T>(c, x, (size_t)nrhs * n);
  copy<T>(c, r, b, (size_t)nrhs * n);
  std::vector<int> it(nrhs, 0), kk(nrhs), act(nrhs);
  bool all_conv = true;
  for (int cyc = 0; cyc <= max_restarts; ++cyc) {
    bool any = false;
    for (int k = 0; k < nrhs; ++k) any = any || (bn[k] > 0 && beta[k] > tol * bn[k]);
    if (!any) break;
    // S.nrm2 holds ||r_k||^2 here
    launch_arnoldi_start(nrhs, m, S.nrm2, S.bn, tol, S.g, S.active, S.kk, S.coef, c->st);
    launch_scale<T>(S.coef, r, n, Vb, n, n, nrhs, false, c->st);
    // one Arnoldi step: w = A M v_j orthogonalised (CGS twice), Givens update
    auto step = [&](int j) {
      cplx<T> *vj = Vb + j * vs, *w = Vb + (j + 1) * vs;
      const cplx<T> *src = vj;
      if (flex) {
        ops.precond(vj, Zb + j * vs);
        src = Zb + j * vs;
      }
      ops.apply(src, w);
      launch_dots<T>(j + 1, Vb, vs, n, w, n, n, nrhs, S.h1, sc, c->st, S.active);
      launch_multi_axpy<T>(j + 1, Vb, vs, n, S.h1, w, n, n, nrhs, -1.0, c->st, S.active);
      launch_dots<T>(j + 1, Vb, vs, n, w, n, n, nrhs, S.h2, sc, c->st, S.active);
      launch_multi_axpy<T>(j + 1, Vb, vs, n, S.h2, w, n, n, nrhs, -1.0, c->st, S.active);
      launch_dots<T>(1, w, 0, n, w, n, n, nrhs, S.nrm2, sc, c->st, S.active);
      launch_arnoldi_update(j, m, nrhs, S.h1, S.h2, S.nrm2, S.H, S.cs, S.sn, S.g, S.bn, tol, S.active, S.kk, S.coef,
                            S.bad, c->st);
      launch_scale<T>(S.coef, w, n, w, n, n, nrhs, false, c->st);
    };
    for (int j = 0; j < m; ++j) {
      if (check_every > 0 && j > 0 && j % check_every == 0) {
        LQ_HIP(hipMemcpyAsync(act.data(), S.active, nrhs * sizeof(int), hipMemcpyDeviceToHost, c->st));
        sync(c);
        bool run = false;
        for (int k = 0; k < nrhs; ++k) run = run || act[k];
        if (!run) break;
      }
      if (graph_id && check_every > 0) {
        // steps j .. j + len - 1, up to the next check
        const int j0 = j, len = std::min(check_every - j % check_every, m - j);
        std::vector<uint64_t> key = *graph_id;
        key.insert(key.end(), {(uint64_t)sizeof(T), (uint64_t)n, (uint64_t)nrhs, (uint64_t)m, (uint64_t)j0,
                               (uint64_t)len, key_bits(tol), key_bits(Vb), key_bits(Zb), key_bits(sc),
                               key_bits(S.h1), key_bits(S.h2), key_bits(S.nrm2), key_bits(S.H), key_bits(S.cs),
                               key_bits(S.sn), key_bits(S.g), key_bits(S.bn), key_bits(S.active), key_bits(S.kk),
                               key_bits(S.coef), key_bits(S.bad)});
        hipGraphExec_t ex = chunk_graph(c, key, [&] {
          for (int jj = j0; jj < j0 + len; ++jj) step(jj);
        });
        LQ_HIP(hipGraphLaunch(ex, c->st));
        j += len - 1;
        continue;
      }
      step(j);
    }
    // x += sum_i y_i (Z_i or V_i)
    launch_arnoldi_solve(m, nrhs, S.H, S.g, S.kk, S.Y, c->st);
    launch_multi_axpy<T>(m, flex ? Zb : Vb, vs, n, S.Y, x, n, n, nrhs, 1.0, c->st);
    ops.resid(b, x, r);
    launch_dots<T>(1, r, 0, n, r, n, n, nrhs, S.nrm2, sc, c->st);
    LQ_HIP(hipMemcpyAsync(h_nrm.data(), S.nrm2, nrhs * sizeof(c128), hipMemcpyDeviceToHost, c->st));
    LQ_HIP(hipMemcpyAsync(kk.data(), S.kk, nrhs * sizeof(int), hipMemcpyDeviceToHost, c->st));
    int bad = 0;
    LQ_HIP(hipMemcpyAsync(&bad, S.bad, sizeof(int), hipMemcpyDeviceToHost, c->st));
    sync(c);
    if (bad) fail(LQ_ERR_NUMERIC, "non-finite Krylov vector");
    for (int k = 0; k < nrhs; ++k) {
      beta[k] = std::sqrt(std::max(0.0, h_nrm[k].re));
      if (!std::isfinite(beta[k])) fail(LQ_ERR_NUMERIC, "non-finite residual");
      it[k] += kk[k];
    }
  }
  for (int k = 0; k < nrhs; ++k) {
    const double rr = bn[k] > 0 ? beta[k] / bn[k] : 0.0;
    if (iters) iters[k] = it[k];
    if (relres) relres[k] = rr;
    if (rr > tol) all_conv = false;
  }
  return all_conv;
}

// ---------------------------------------------------------------------------
// multigrid pieces in precision T
// ---------------------------------------------------------------------------
template <typename T> MGData<T> &mgd(lq_ctx *c);
template <> MGData<double> &mgd<double>(lq_ctx *c) { return c->d64; }
template <> MGData<float> &mgd<float>(lq_ctx *c) { return c->d32; }
// The clover term to pass with the links (nullptr without one): canonical
// FP64 / FP32 for the caller's links, blocked FP64 for the outer operator,
// blocked in the multigrid's precision.
const c128 *clov_can(lq_ctx *c) { return c->csw != 0 ? c->clov_can.p : nullptr; }
const c64 *clov_can32(lq_ctx *c) { return c->csw != 0 ? c->clov_can32.p : nullptr; }
const c128 *clov_blk(lq_ctx *c) { return c->csw != 0 ? c->clov64.p : nullptr; }
template <typename T> const cplx<T> *clov_mg(lq_ctx *c) { return c->csw != 0 ? mgd<T>(c).C.p : nullptr; }

template <typename T> KrylovWork<T> &ckw(lq_ctx *c);
template <> KrylovWork<double> &ckw<double>(lq_ctx *c) { return c->coarse_kw64; }
template <> KrylovWork<float> &ckw<float>(lq_ctx *c) { return c->coarse_kw32; }

Shifts shifts_of(const double *s, int n) {
  Shifts S;
  for (int k = 0; k < kMaxRhs; ++k) S.s[k] = (k < n && s) ? s[k] : 0.0;
  return S;
}

// z = SAP steps on (Q - sigma) z = r, continuing from the current z
template <typename T>
void sap(lq_ctx *c, const double *sig, const cplx<T> *r, cplx<T> *z, int nrhs, int steps) {
  Shifts S = shifts_of(sig, nrhs);
  for (int s = 0; s < steps; ++s)
    for (int col = 0; col < 2; ++col)
      if (c->nblocks[col] > 0)
        launch_sap_colour<T>(c->g, mgd<T>(c).U.p, r, z, c->blocks[col].p, c->nblocks[col], c->m0, S, nrhs,
                             c->p.sap_mr, c->st, clov_mg<T>(c));
}

// Restarted GMRES for (Q_c - sigma) e = c on one coarse level (the operator
// cg / Qc), run on the equivalent gamma5^c form (R16: same solution, a field
// of values near the right half plane).  QcB: the bfloat16 copy of an FP32
// operator, or null.  graphs: the Arnoldi chunks may be replayed from
// captured graphs (direct launches otherwise).
template <typename T>
void coarse_gmres(lq_ctx *c, const CoarseGeom &cg, const cplx<T> *Qc, const bf16c *QcB, KrylovWork<T> &kw,
                  const double *sig, const cplx<T> *rc, cplx<T> *ec, int nrhs, cplx<T> *rhs_buf, int m, int restarts,
                  double tol, bool graphs_ok) {
  const long long n = (long long)cg.nA * cg.n2;
  Shifts S = shifts_of(sig, nrhs);
  launch_coarse_g5<T>(cg, rc, rhs_buf, nrhs, c->st);
  // graphs only while the coarse apply is not being timed (its timed launch
  // records events, which a capture cannot hold).  With graphs the shifts go
  // to device memory, so the coarse-apply launches are the same for every
  // solve of this shape and the captured steps can be replayed.
  const bool graphs = graphs_ok && c->p.graphs && g_ktimer_class != KT_COARSE;
  double *dsig = nullptr;
  if (graphs) {
    dsig = c->coarse_sig.get(kMaxRhs);
    launch_set_shifts(S, nrhs, dsig, c->st);
  }
  KOps<T> ops;
  auto capply = [=](const cplx<T> *x, cplx<T> *y) {
    if constexpr (std::is_same<T, float>::value) {
      if (QcB) {
        launch_coarse_apply_bf16(cg, QcB, x, y, S, nrhs, true, c->st, dsig);
        return;
      }
    }
    launch_coarse_apply<T>(cg, Qc, x, y, S, nrhs, true, c->st, dsig);
  };
  // kernel variant for this shape: timed once, before any capture (ec is
  // overwritten here and zeroed by GMRES)
  int variant;
  if constexpr (std::is_same<T, float>::value)
    variant = QcB ? tune_coarse_apply_bf16(cg, QcB, rhs_buf, ec, nrhs, c->st)
                  : tune_coarse_apply<T>(cg, Qc, rhs_buf, ec, nrhs, c->st);
  else
    variant = tune_coarse_apply<T>(cg, Qc, rhs_buf, ec, nrhs, c->st);
  ops.apply = capply;
  const c128 *pm1 = c->minus_one.p, *pp1 = c->plus_one.p;
  ops.resid = [=](const cplx<T> *b, const cplx<T> *x, cplx<T> *r) {
    capply(x, r);
    launch_scale<T>(pm1, r, n, r, n, n, nrhs, false, c->st);                 // r = -A x
    launch_multi_axpy<T>(1, b, 0, n, pp1, r, n, n, nrhs, 1.0, c->st);       // r += b
  };
  int its[kMaxRhs];
  // every by-value argument of the captured launches belongs to the key: the
  // coarse lattice extents too (two aggregate shapes with equal nA and n2 must
  // not share a graph)
  const std::vector<uint64_t> gid = {QcB ? key_bits(QcB) : key_bits(Qc), key_bits(dsig), (uint64_t)cg.nA,
                                     (uint64_t)cg.n2, (uint64_t)cg.nb[0], (uint64_t)cg.nb[1],
                                     (uint64_t)cg.nb[2], (uint64_t)cg.nb[3],
                                     (uint64_t)variant, key_bits(pm1)};
  gmres_batched<T>(c, kw, n, nrhs, ops, rhs_buf, ec, m, restarts, tol, its, nullptr, 8, graphs ? &gid : nullptr);
  for (int k = 0; k < nrhs; ++k) c->coarse_iters += its[k];
}

template <typename T> KrylovWork<T> &s1kw(lq_ctx *c);
template <> KrylovWork<double> &s1kw<double>(lq_ctx *c) { return c->smooth1_kw64; }
template <> KrylovWork<float> &s1kw<float>(lq_ctx *c) { return c->smooth1_kw32; }
template <typename T> KrylovWork<T> &c2kw(lq_ctx *c);
template <> KrylovWork<double> &c2kw<double>(lq_ctx *c) { return c->coarse2_kw64; }
template <> KrylovWork<float> &c2kw<float>(lq_ctx *c) { return c->coarse2_kw32; }
template <typename T> cplx<T> *l1work(lq_ctx *c, size_t n);
template <> c128 *l1work<double>(lq_ctx *c, size_t n) { return c->l1w64.get(n); }
template <> c64 *l1work<float>(lq_ctx *c, size_t n) { return c->l1w32.get(n); }
template <typename T> cplx<T> *l2work(lq_ctx *c, size_t n);
template <> c128 *l2work<double>(lq_ctx *c, size_t n) { return c->l2w64.get(n); }
template <> c64 *l2work<float>(lq_ctx *c, size_t n) { return c->l2w32.get(n); }

// The level-1 two-grid cycle B1 ~ (Q_c - sigma)^{-1} of the three-level
// hierarchy: the level-2 correction P2 (Q_c2 - sigma)^{-1} P2^dag r (GMRES to
// coarse2_tol), then post1 smoothing steps, each smooth1_m GMRES steps on
// gamma5^c (Q_c - sigma) for the current residual.
template <typename T>
void cycle1(lq_ctx *c, const double *sig, const cplx<T> *r1, cplx<T> *z1, int nrhs) {
  const long long n1 = (long long)c->cg.nA * c->cg.n2, n2 = (long long)c->cg2.nA * c->cg2.n2;
  auto &d = mgd<T>(c);
  Shifts S = shifts_of(sig, nrhs);
  cplx<T> *w2 = l2work<T>(c, (size_t)3 * kMaxRhs * n2);
  cplx<T> *r2 = w2, *e2 = w2 + kMaxRhs * n2, *b2 = w2 + 2 * kMaxRhs * n2;
  cplx<T> *w1 = l1work<T>(c, (size_t)3 * kMaxRhs * n1);
  cplx<T> *t1 = w1, *g1 = w1 + kMaxRhs * n1, *d1 = w1 + 2 * kMaxRhs * n1;
  launch_restrict2<T>(c->l2g, d.P2.p, r1, nrhs, r2, c->st);
  if (c->p.coarse2_tol > 0) {
    coarse_gmres<T>(c, c->cg2, d.Qc2.p, nullptr, c2kw<T>(c), sig, r2, e2, nrhs, b2, c->p.coarse2_m,
                    c->p.coarse2_restarts, c->p.coarse2_tol, false);
  } else {
    // coarse2_tol = 0: a fixed number (coarse2_m) of GMRES steps on the
    // gamma5^c2 form, without host reads
    const CoarseGeom cg2 = c->cg2;
    const cplx<T> *Qc2 = d.Qc2.p;
    launch_coarse_g5<T>(cg2, r2, b2, nrhs, c->st);
    KOps<T> ops2;
    ops2.apply = [=](const cplx<T> *x, cplx<T> *y) { launch_coarse_apply<T>(cg2, Qc2, x, y, S, nrhs, true, c->st); };
    zero<T>(c, e2, (size_t)nrhs * n2);
    gmres_fixed<T>(c, c2kw<T>(c), n2, nrhs, ops2, b2, e2, c->p.coarse2_m);
  }
  launch_prolong2<T>(c->l2g, d.P2.p, e2, z1, nrhs, false, c->st);
  const c128 *pm1 = c->minus_one.p, *pp1 = c->plus_one.p;
  for (int step = 0; step < c->p.post1; ++step) {
    // g1 = gamma5^c (r1 - (Q_c - sigma) z1)
    launch_coarse_apply<T>(c->cg, d.Qc.p, z1, t1, S, nrhs, false, c->st);
    launch_scale<T>(pm1, t1, n1, t1, n1, n1, nrhs, false, c->st);
    launch_multi_axpy<T>(1, r1, 0, n1, pp1, t1, n1, n1, nrhs, 1.0, c->st);
    launch_coarse_g5<T>(c->cg, t1, g1, nrhs, c->st);
    KOps<T> ops;
    const CoarseGeom cg = c->cg;
    const cplx<T> *Qc = d.Qc.p;
    ops.apply = [=](const cplx<T> *x, cplx<T> *y) { launch_coarse_apply<T>(cg, Qc, x, y, S, nrhs, true, c->st); };
    ops.resid = [=](const cplx<T> *b, const cplx<T> *x, cplx<T> *r) {
      launch_coarse_apply<T>(cg, Qc, x, r, S, nrhs, true, c->st);
      launch_scale<T>(pm1, r, n1, r, n1, n1, nrhs, false, c->st);
      launch_multi_axpy<T>(1, b, 0, n1, pp1, r, n1, n1, nrhs, 1.0, c->st);
    };
    zero<T>(c, d1, (size_t)nrhs * n1);
    gmres_fixed<T>(c, s1kw<T>(c), n1, nrhs, ops, g1, d1, c->p.smooth1_m);
    launch_multi_axpy<T>(1, d1, 0, n1, pp1, z1, n1, n1, nrhs, 1.0, c->st);
  }
}

// The coarse solve of the cycle: two levels, restarted GMRES on Q_c; three
// levels, FGMRES on Q_c - sigma right-preconditioned by the level-1 cycle.
template <typename T>
void coarse_solve(lq_ctx *c, const double *sig, const cplx<T> *rc, cplx<T> *ec, int nrhs, cplx<T> *rhs_buf) {
  const cplx<T> *Qc = mgd<T>(c).Qc.p;
  if (c->n_levels == 2) {
    // the FP32 cycle may read Q_c from its bfloat16 copy (FP32 arithmetic)
    const bf16c *QcB = nullptr;
    if constexpr (std::is_same<T, float>::value)
      if (c->p.coarse_bf16) QcB = c->QcB.p;
    coarse_gmres<T>(c, c->cg, Qc, QcB, ckw<T>(c), sig, rc, ec, nrhs, rhs_buf, c->p.coarse_m, c->p.coarse_restarts,
                    c->p.coarse_tol, true);
    return;
  }
  const long long n1 = (long long)c->cg.nA * c->cg.n2;
  Shifts S = shifts_of(sig, nrhs);
  std::vector<double> sv(sig, sig + nrhs);
  const CoarseGeom cg = c->cg;
  const c128 *pm1 = c->minus_one.p, *pp1 = c->plus_one.p;
  KOps<T> ops;
  ops.apply = [=](const cplx<T> *x, cplx<T> *y) { launch_coarse_apply<T>(cg, Qc, x, y, S, nrhs, false, c->st); };
  ops.precond = [=](const cplx<T> *v, cplx<T> *z) { cycle1<T>(c, sv.data(), v, z, nrhs); };
  ops.resid = [=](const cplx<T> *b, const cplx<T> *x, cplx<T> *r) {
    launch_coarse_apply<T>(cg, Qc, x, r, S, nrhs, false, c->st);
    launch_scale<T>(pm1, r, n1, r, n1, n1, nrhs, false, c->st);
    launch_multi_axpy<T>(1, b, 0, n1, pp1, r, n1, n1, nrhs, 1.0, c->st);
  };
  int its[kMaxRhs];
  gmres_batched<T>(c, ckw<T>(c), n1, nrhs, ops, rc, ec, c->p.coarse_m, c->p.coarse_restarts, c->p.coarse_tol, its,
                   nullptr, 1);
  for (int k = 0; k < nrhs; ++k) c->coarse_iters += its[k];
}

template <typename T> struct CycleBufs { cplx<T> *tmp, *rc, *ec, *cb; };

template <typename T> CycleBufs<T> cycle_bufs(lq_ctx *c, int nrhs);
template <> CycleBufs<double> cycle_bufs<double>(lq_ctx *c, int nrhs) {
  const size_t nf = (size_t)nrhs * 12 * c->g.V, nc = (size_t)nrhs * c->cg.nA * c->cg.n2;
  c128 *cbuf = c->c64a.get(3 * nc);
  return {c->f64a.get(nf), cbuf, cbuf + nc, cbuf + 2 * nc};
}
template <> CycleBufs<float> cycle_bufs<float>(lq_ctx *c, int nrhs) {
  const size_t nf = (size_t)nrhs * 12 * c->g.V, nc = (size_t)nrhs * c->cg.nA * c->cg.n2;
  c64 *cbuf = c->c32a.get(3 * nc);
  return {c->f32c.get(nf), cbuf, cbuf + nc, cbuf + 2 * nc};
}

// z = B_sigma r: one multigrid cycle (eq. E_2g) in precision T.
template <typename T>
void cycle(lq_ctx *c, const double *sig, const cplx<T> *r, cplx<T> *z, int nrhs) {
  const size_t nf = (size_t)nrhs * 12 * c->g.V;
  CycleBufs<T> b = cycle_bufs<T>(c, nrhs);
  auto &d = mgd<T>(c);
  zero<T>(c, z, nf);
  const cplx<T> *rr = r;
  if (c->p.pre > 0) {
    sap<T>(c, sig, r, z, nrhs, c->p.pre);
    launch_wilson<T>(c->g, d.U.p, z, b.tmp, r, c->m0, shifts_of(sig, nrhs), nrhs, W_RESID, c->st, clov_mg<T>(c));
    rr = b.tmp;
  }
  launch_restrict<T>(c->g, d.P.p, c->Nv, rr, 12LL * c->g.V, nrhs, b.rc, c->st);
  coarse_solve<T>(c, sig, b.rc, b.ec, nrhs, b.cb);
  launch_prolong<T>(c->g, d.P.p, c->Nv, b.ec, z, 12LL * c->g.V, nrhs, true, c->st);
  if (c->p.post > 0) sap<T>(c, sig, r, z, nrhs, c->p.post);
}

// z = B_sigma v with FP64 input/output; the cycle runs in the configured precision.
void precond64(lq_ctx *c, const double *sig, const c128 *v, c128 *z, int nrhs) {
  if (c->p.precision == LQ_PREC_FP64) {
    cycle<double>(c, sig, v, z, nrhs);
  } else {
    const size_t nf = (size_t)nrhs * 12 * c->g.V;
    c64 *v32 = c->f32a.get(nf), *z32 = c->f32b.get(nf);
    launch_convert<float, double>(v, v32, (long long)nf, c->st);
    cycle<float>(c, sig, v32, z32, nrhs);
    launch_convert<double, float>(z32, z, (long long)nf, c->st);
  }
}

// smoother only (FP64 interface), from z = 0
void smooth64(lq_ctx *c, const double *sig, const c128 *r, c128 *z, int nrhs, int steps) {
  const size_t nf = (size_t)nrhs * 12 * c->g.V;
  if (c->p.precision == LQ_PREC_FP64) {
    zero<double>(c, z, nf);
    sap<double>(c, sig, r, z, nrhs, steps);
  } else {
    c64 *r32 = c->f32a.get(nf), *z32 = c->f32b.get(nf);
    launch_convert<float, double>(r, r32, (long long)nf, c->st);
    zero<float>(c, z32, nf);
    sap<float>(c, sig, r32, z32, nrhs, steps);
    launch_convert<double, float>(z32, z, (long long)nf, c->st);
  }
}

// Q_c = P^dag Q P in precision T from P_T and U_T.
template <typename T> void build_coarse(lq_ctx *c, DevBuf<cplx<T>> &parts, DevBuf<cplx<T>> &pc) {
  auto &d = mgd<T>(c);
  const int Nv = c->Nv, n2 = 2 * Nv, nA = c->cg.nA;
  const long long V12 = 12LL * c->g.V;
  const int C = std::min(Nv, 4);           // columns per pass: 5*C split-hop fields in flight
  cplx<T> *pa = parts.get((size_t)C * 5 * V12);
  cplx<T> *pcb = pc.get((size_t)C * 5 * nA * n2);
  cplx<T> *Qc = d.Qc.get((size_t)nA * 5 * n2 * n2);
  int *dint = c->ints.get(2 * C);
  for (int h = 0; h < 2; ++h)
    for (int l0 = 0; l0 < Nv; l0 += C) {
      const int nc = std::min(C, Nv - l0);
      std::vector<int> hi(2 * C);
      for (int j = 0; j < nc; ++j) { hi[j] = h; hi[C + j] = h * Nv + l0 + j; }
      LQ_HIP(hipMemcpyAsync(dint, hi.data(), 2 * C * sizeof(int), hipMemcpyHostToDevice, c->st));
      launch_coarse_parts<T>(c->g, d.U.p, d.P.p + l0 * V12, dint, nc, V12, pa, c->m0, c->st, clov_mg<T>(c));
      launch_restrict<T>(c->g, d.P.p, Nv, pa, V12, 5 * nc, pcb, c->st);
      launch_scatter_coarse<T>(pcb, nc, dint + C, n2, nA, Qc, c->st);
      sync(c);
    }
}

// Q_c2 = P2^dag Q_c P2 in precision T from P2_T and Q_c (T): the split
// couplings of Q_c applied to each half-column of P2, restricted, scattered.
template <typename T> void build_coarse2(lq_ctx *c, DevBuf<cplx<T>> &parts, DevBuf<cplx<T>> &pc) {
  auto &d = mgd<T>(c);
  const int Nv2 = c->Nv2, n22 = 2 * Nv2, nA2 = c->cg2.nA;
  const long long n1 = (long long)c->cg.nA * c->cg.n2;
  const int C = std::min(Nv2, 3);          // 5 C <= 16 restricted parts per pass
  cplx<T> *pa = parts.get((size_t)C * 5 * n1);
  cplx<T> *pcb = pc.get((size_t)C * 5 * nA2 * n22);
  cplx<T> *Qc2 = d.Qc2.get((size_t)nA2 * 5 * n22 * n22);
  int *dint = c->ints.get(2 * C);
  for (int h = 0; h < 2; ++h)
    for (int l0 = 0; l0 < Nv2; l0 += C) {
      const int nc = std::min(C, Nv2 - l0);
      std::vector<int> hi(2 * C);
      for (int j = 0; j < nc; ++j) { hi[j] = h; hi[C + j] = h * Nv2 + l0 + j; }
      LQ_HIP(hipMemcpyAsync(dint, hi.data(), 2 * C * sizeof(int), hipMemcpyHostToDevice, c->st));
      launch_coarse_parts2<T>(c->l2g, d.Qc.p, d.P2.p + l0 * n1, dint, nc, n1, pa, c->st);
      launch_restrict2<T>(c->l2g, d.P2.p, pa, 5 * nc, pcb, c->st);
      launch_scatter_coarse<T>(pcb, nc, dint + C, n22, nA2, Qc2, c->st);
      sync(c);
    }
}

// The third level from the first Nv2 of the fields src (blocked FP64) that
// built P: their restrictions P^dag src are the level-1 test vectors of P2
// (the level-1 images of the approximations, as the fine vectors are for P).
// Dependence on a level-2 aggregate half: an error, or with keep_dependent
// that block of P2 keeps its previous columns (returns false).
bool rebuild2(lq_ctx *c, const std::vector<const c128 *> &src, bool keep_dependent) {
  const long long V12 = 12LL * c->g.V, n1 = (long long)c->cg.nA * c->cg.n2;
  const size_t nP2 = (size_t)c->Nv2 * n1;
  c128 *W2 = c->W2.get(nP2);
  // restriction with the FP64 P, one field per launch (the fields need not be contiguous)
  for (int k = 0; k < c->Nv2; ++k) launch_restrict<double>(c->g, c->P64.p, c->Nv, src[k], V12, 1, W2 + k * n1, c->st);
  int *st = c->status.get(1);
  LQ_HIP(hipMemsetAsync(st, 0, sizeof(int), c->st));
  c128 *P2 = c->P2_64.get(nP2);
  launch_build_P2(c->l2g, W2, P2, st, c->st);
  int h_st = 0;
  LQ_HIP(hipMemcpyAsync(&h_st, st, sizeof(int), hipMemcpyDeviceToHost, c->st));
  sync(c);
  if (h_st && !keep_dependent) fail(LQ_ERR_NUMERIC, "level-1 test vectors are linearly dependent on a level-2 aggregate");
  if (c->p.precision == LQ_PREC_FP64) {
    copy<double>(c, c->d64.P2.get(nP2), P2, nP2);
    build_coarse2<double>(c, c->parts2_64, c->pc2_64);
  } else {
    launch_convert<float, double>(P2, c->d32.P2.get(nP2), (long long)nP2, c->st);
    build_coarse2<float>(c, c->parts2_32, c->pc2_32);
  }
  sync(c);
  return h_st == 0;
}

// P and Q_c from the FP64 fields src [Nv][12][V] (blocked).  Fields that are
// linearly dependent on some aggregate half are an error, unless keep_dependent:
// then those blocks of P keep their previous columns (the other blocks are
// rebuilt, P stays orthonormal and gamma5-split) and the call returns false.
bool rebuild(lq_ctx *c, const std::vector<const c128 *> &src, bool keep_dependent = false) {
  const size_t nP = (size_t)c->Nv * 12 * c->g.V;
  if ((int)src.size() != c->Nv) fail(LQ_ERR_ARG, "rebuild: need Nv source fields");
  int *st = c->status.get(1);
  LQ_HIP(hipMemsetAsync(st, 0, sizeof(int), c->st));
  c128 *P64 = c->P64.get(nP);
  const c128 **cols = c->src_cols.get(src.size());
  LQ_HIP(hipMemcpyAsync(cols, src.data(), src.size() * sizeof(const c128 *), hipMemcpyHostToDevice, c->st));
  launch_build_P(c->g, cols, c->Nv, P64, st, c->st);
  int h_st = 0;
  LQ_HIP(hipMemcpyAsync(&h_st, st, sizeof(int), hipMemcpyDeviceToHost, c->st));
  sync(c);
  if (h_st && !keep_dependent) fail(LQ_ERR_NUMERIC, "test vectors are linearly dependent on an aggregate");
  if (c->p.precision == LQ_PREC_FP64) {
    copy<double>(c, c->d64.P.get(nP), P64, nP);
    build_coarse<double>(c, c->parts64, c->pc64);
  } else {
    launch_convert<float, double>(P64, c->d32.P.get(nP), (long long)nP, c->st);
    build_coarse<float>(c, c->parts32, c->pc32);
    if (c->p.coarse_bf16) {
      const long long nq = (long long)c->cg.nA * 5 * c->cg.n2 * c->cg.n2;
      launch_to_bf16(c->d32.Qc.p, c->QcB.get((size_t)nq), nq, c->st);
    }
  }
  sync(c);
  bool ok2 = true;
  if (c->n_levels == 3) ok2 = rebuild2(c, src, keep_dependent);
  return h_st == 0 && ok2;
}

// Addresses of n consecutive fields starting at F.
std::vector<const c128 *> fields_of(const lq_ctx *c, const c128 *F, int n) {
  std::vector<const c128 *> v(n);
  for (int k = 0; k < n; ++k) v[k] = F + (long long)k * 12 * c->g.V;
  return v;
}

// Gram-Schmidt (twice) of n fields in place, in index order; FP64.
void orthonormalise(lq_ctx *c, c128 *F, int n) {
  const long long L = 12LL * c->g.V;
  for (int k = 0; k < n; ++k) {
    for (int pass = 0; pass < 2; ++pass) {
      auto h = dots<double>(c, k, F, L, 0, F + k * L, 0, L, 1);
      axpys<double>(c, k, F, L, 0, h, F + k * L, 0, L, 1, -1.0);
    }
    auto nr = norms<double>(c, F + k * L, L, 1);
    if (!(nr[0] > 0) || !std::isfinite(nr[0])) fail(LQ_ERR_NUMERIC, "vector collapsed in Gram-Schmidt");
    scale<double>(c, std::vector<cd>{cd(1.0 / nr[0])}, F + k * L, 0, F + k * L, 0, L, 1, false);
  }
}

// FGMRES for (Q - sigma_k) x_k = b_k, FP64, blocked layout.
struct Deflation;
void deflated_precond(lq_ctx *c, const Deflation &D, const double *sig, const c128 *in, c128 *out, int nrhs);

bool solve_shifted(lq_ctx *c, int nrhs, const double *sig, const c128 *b, c128 *x, double tol, int *iters,
                   double *relres, int max_restarts, const Deflation *D = nullptr) {
  const long long n = 12LL * c->g.V;
  Shifts S = shifts_of(sig, nrhs);
  std::vector<double> sv(sig, sig + nrhs);
  KOps<double> ops;
  ops.apply = [=](const c128 *in, c128 *out) {
    launch_wilson<double>(c->g, c->U64.p, in, out, nullptr, c->m0, S, nrhs, W_QSHIFT, c->st, clov_blk(c));
  };
  if (D)
    ops.precond = [=](const c128 *in, c128 *out) { deflated_precond(c, *D, sv.data(), in, out, nrhs); };
  else
    ops.precond = [=](const c128 *in, c128 *out) { precond64(c, sv.data(), in, out, nrhs); };
  ops.resid = [=](const c128 *bb, const c128 *xx, c128 *r) {
    launch_wilson<double>(c->g, c->U64.p, xx, r, bb, c->m0, S, nrhs, W_RESID, c->st, clov_blk(c));
  };
  return gmres_batched<double>(c, c->fine_kw, n, nrhs, ops, b, x, c->p.fgmres_m, max_restarts, tol, iters, relres,
                               1);
}

// Hermitian eigensolver: Householder reduction to tridiagonal form, a diagonal
// phase change that makes the tridiagonal real, and the implicit QL iteration
// with Wilkinson shifts.  On return A = diag(eigenvalues) (real parts on the
// diagonal) and Vm holds the orthonormal eigenvectors as columns (row-major).
void herm_eigh(int n, std::vector<cd> &A, std::vector<cd> &Vm) {
  auto a = [&](int i, int j) -> cd & { return A[(size_t)i * n + j]; };
  Vm.assign((size_t)n * n, cd(0));
  auto q = [&](int i, int j) -> cd & { return Vm[(size_t)i * n + j]; };
  for (int i = 0; i < n; ++i) q(i, i) = 1.0;
  std::vector<cd> v(n), p(n), w(n);
  // 1. A <- H A H with H = 1 - 2 v v^dag zeroing column k below the subdiagonal
  for (int k = 0; k + 2 < n; ++k) {
    double xn = 0;
    for (int i = k + 1; i < n; ++i) xn += std::norm(a(i, k));
    xn = std::sqrt(xn);
    if (xn == 0) continue;
    const cd x0 = a(k + 1, k);
    const cd ph = (std::abs(x0) > 0) ? x0 / std::abs(x0) : cd(1.0);
    const cd alpha = -ph * xn;
    double vn = 0;
    for (int i = k + 1; i < n; ++i) {
      v[i] = a(i, k) - (i == k + 1 ? alpha : cd(0));
      vn += std::norm(v[i]);
    }
    vn = std::sqrt(vn);
    if (vn == 0) continue;
    for (int i = k + 1; i < n; ++i) v[i] /= vn;
    // full rows/cols k..n-1 take part: p = A v over the trailing block (column k included)
    for (int i = k; i < n; ++i) {
      cd s = 0;
      for (int j = k + 1; j < n; ++j) s += a(i, j) * v[j];
      p[i] = s;
    }
    double K = 0;
    for (int i = k + 1; i < n; ++i) K += (std::conj(v[i]) * p[i]).real();
    // w = p - K v (v zero at index k)
    for (int i = k; i < n; ++i) w[i] = p[i] - (i > k ? K * v[i] : cd(0));
    // A <- A - 2 (v w^dag + w v^dag) on rows/cols k..n-1
    for (int i = k; i < n; ++i) {
      const cd vi = (i > k) ? v[i] : cd(0), wi = w[i];
      for (int j = k; j < n; ++j) {
        const cd vj = (j > k) ? v[j] : cd(0);
        a(i, j) -= 2.0 * (vi * std::conj(w[j]) + wi * std::conj(vj));
      }
    }
    // Q <- Q H
    for (int i = 0; i < n; ++i) {
      cd s = 0;
      for (int j = k + 1; j < n; ++j) s += q(i, j) * v[j];
      for (int j = k + 1; j < n; ++j) q(i, j) -= 2.0 * s * std::conj(v[j]);
    }
  }
  // 2. real tridiagonal: d_i = A_ii, e_i = |A_{i+1,i}|; phases into Q's columns
  std::vector<double> d(n), e(n, 0.0);
  cd phi = 1.0;
  for (int i = 0; i < n; ++i) {
    d[i] = a(i, i).real();
    if (i > 0) {
      const cd sub = a(i, i - 1);
      const double r = std::abs(sub);
      if (r > 0) phi *= sub / r;
      for (int k = 0; k < n; ++k) q(k, i) *= phi;
      e[i - 1] = r;
    }
  }
  // 3. implicit QL with Wilkinson shifts; rotations applied to Q's columns
  for (int l = 0; l < n; ++l) {
    for (int iter = 0; iter < 60; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 1e-16 * dd) break;
      }
      if (m == l) break;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + (g >= 0 ? r : -r));
      double s = 1, c = 1, pp = 0;
      int i = m - 1;
      for (; i >= l; --i) {
        double f = s * e[i], b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0) {
          d[i + 1] -= pp;
          e[m] = 0;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - pp;
        r = (d[i] - g) * s + 2.0 * c * b;
        pp = s * r;
        d[i + 1] = g + pp;
        g = c * r - b;
        for (int k = 0; k < n; ++k) {
          const cd t = q(k, i + 1);
          q(k, i + 1) = s * q(k, i) + c * t;
          q(k, i) = c * q(k, i) - s * t;
        }
      }
      if (r == 0 && i >= l) continue;
      d[l] -= pp;
      e[l] = g;
      e[m] = 0;
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a(i, j) = (i == j) ? cd(d[i]) : cd(0);
}

// Rayleigh-Ritz on span(E) (E orthonormal, n fields): H = E^dag Q E, H = C w C^dag,
// E <- E C ordered by (|w|, w); lam receives w.

// Reorder the n fields of E in place so that slot p receives old slot order[p]
// (cycle following with one spare field).
void permute_fields(lq_ctx *c, c128 *E, const std::vector<int> &order, c128 *spare) {
  const long long V12 = 12LL * c->g.V;
  const int n = (int)order.size();
  std::vector<char> done(n, 0);
  for (int p = 0; p < n; ++p) {
    if (done[p] || order[p] == p) { done[p] = 1; continue; }
    copy<double>(c, spare, E + p * V12, V12);
    int cur = p;
    while (true) {
      const int src = order[cur];
      done[cur] = 1;
      if (src == p) { copy<double>(c, E + cur * V12, spare, V12); break; }
      copy<double>(c, E + cur * V12, E + src * V12, V12);
      cur = src;
    }
  }
  sync(c);
}

// Rayleigh-Ritz on the trailing fields E[L..n) (the unconverged vectors; the
// converged ones sit in E[0..L)).  The trailing block is first projected
// against E[0..L) (block Gram-Schmidt, twice); then with H = E_U^dag Q E_U and
// G = E_U^dag E_U the pencil (H, G) is reduced by G = L L^dag to
// L^-1 H L^-dag = Z w Z^dag, and the Ritz vectors E_U L^-dag Z, ordered by
// (|w|, w), replace E_U.  spill[j] is room for Ritz vector j (n - L fields,
// none overlapping E).
void rayleigh_ritz_tail(lq_ctx *c, c128 *E, int n, int L, std::vector<double> &lam,
                        const std::vector<c128 *> &spill) {
  const long long V12 = 12LL * c->g.V;
  const int m = n - L;
  c128 *EU = E + (long long)L * V12;
  for (int pass = 0; pass < 2 && L > 0; ++pass)
    for (int j0 = 0; j0 < m; j0 += kMaxRhs) {
      const int nk = std::min(kMaxRhs, m - j0);
      auto h = gram(c, L, E, V12, nk, EU + j0 * V12, V12, V12);
      combine(c, L, E, V12, nk, h, -1.0, EU + j0 * V12, V12, V12, true);
    }
  std::vector<cd> H((size_t)m * m), G((size_t)m * m);
  c128 *QE = c->tmpA.get((size_t)kMaxRhs * V12);
  Shifts z = shifts_of(nullptr, 0);
  for (int j0 = 0; j0 < m; j0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, m - j0);
    launch_wilson<double>(c->g, c->U64.p, EU + j0 * V12, QE, nullptr, c->m0, z, nk, W_QSHIFT, c->st, clov_blk(c));
    auto a = gram(c, m, EU, V12, nk, QE, V12, V12);
    auto g = gram(c, m, EU, V12, nk, EU + j0 * V12, V12, V12);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < nk; ++k) {
        H[(size_t)i * m + j0 + k] = a[(size_t)i * nk + k];
        G[(size_t)i * m + j0 + k] = g[(size_t)i * nk + k];
      }
  }
  // Cholesky G = Lc Lc^dag (lower), then M = Lc^-1 H Lc^-dag
  std::vector<cd> Lc((size_t)m * m, cd(0));
  for (int j = 0; j < m; ++j) {
    double d = G[(size_t)j * m + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(Lc[(size_t)j * m + k]);
    if (!(d > 1e-14 * std::fabs(G[(size_t)j * m + j].real()))) fail(LQ_ERR_NUMERIC, "Rayleigh-Ritz basis is singular");
    const double ljj = std::sqrt(d);
    Lc[(size_t)j * m + j] = ljj;
    for (int i = j + 1; i < m; ++i) {
      cd v = G[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) v -= Lc[(size_t)i * m + k] * std::conj(Lc[(size_t)j * m + k]);
      Lc[(size_t)i * m + j] = v / ljj;
    }
  }
  auto lower_solve = [&](std::vector<cd> &B, int ncol) {         // B <- Lc^-1 B, B [m][ncol]
    for (int col = 0; col < ncol; ++col)
      for (int i = 0; i < m; ++i) {
        cd v = B[(size_t)i * ncol + col];
        for (int k = 0; k < i; ++k) v -= Lc[(size_t)i * m + k] * B[(size_t)k * ncol + col];
        B[(size_t)i * ncol + col] = v / Lc[(size_t)i * m + i];
      }
  };
  std::vector<cd> T = H;                  // T = Lc^-1 H
  lower_solve(T, m);
  std::vector<cd> Tt((size_t)m * m);      // Tt = (Lc^-1 T^dag) = Lc^-1 H Lc^-dag (H Hermitian)
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Tt[(size_t)i * m + j] = std::conj(T[(size_t)j * m + i]);
  lower_solve(Tt, m);
  for (int i = 0; i < m; ++i)
    for (int j = i; j < m; ++j) {
      const cd h = 0.5 * (Tt[(size_t)i * m + j] + std::conj(Tt[(size_t)j * m + i]));
      Tt[(size_t)i * m + j] = h;
      Tt[(size_t)j * m + i] = std::conj(h);
    }
  std::vector<cd> Zm;
  herm_eigh(m, Tt, Zm);
  // Y = Lc^-dag Z: back substitution with Lc^dag (upper)
  std::vector<cd> Y = Zm;
  for (int col = 0; col < m; ++col)
    for (int i = m - 1; i >= 0; --i) {
      cd v = Y[(size_t)i * m + col];
      for (int k = i + 1; k < m; ++k) v -= std::conj(Lc[(size_t)k * m + i]) * Y[(size_t)k * m + col];
      Y[(size_t)i * m + col] = v / Lc[(size_t)i * m + i];
    }
  std::vector<int> o(m);
  for (int i = 0; i < m; ++i) o[i] = i;
  std::sort(o.begin(), o.end(), [&](int a, int b) {
    const double wa = Tt[(size_t)a * m + a].real(), wb = Tt[(size_t)b * m + b].real();
    if (std::fabs(wa) != std::fabs(wb)) return std::fabs(wa) < std::fabs(wb);
    return wa < wb;
  });
  c128 *chunk = c->tmpB.get((size_t)kMaxRhs * V12);
  for (int j0 = 0; j0 < m; j0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, m - j0);
    std::vector<cd> h((size_t)m * nk);
    for (int i = 0; i < m; ++i)
      for (int k = 0; k < nk; ++k) h[(size_t)i * nk + k] = Y[(size_t)i * m + o[j0 + k]];
    combine(c, m, EU, V12, nk, h, 1.0, chunk, V12, V12, false);
    for (int k = 0; k < nk; ++k) copy<double>(c, spill[j0 + k], chunk + k * V12, V12);
  }
  for (int j = 0; j < m; ++j) copy<double>(c, EU + (long long)j * V12, spill[j], V12);
  for (int j = 0; j < m; ++j) lam[L + j] = Tt[(size_t)o[j] * m + o[j]].real();
  sync(c);
}


// ---------------------------------------------------------------------------
// Galerkin correction on the span of the current eigenvector approximations.
// With E = [e_1 .. e_n], A = E^dag Q E and G = E^dag E, the correction for
// shift sigma is u = E (A - sigma G)^{-1} E^dag r: the exact solve of (Q - sigma)
// restricted to span(E).  It is applied before the multigrid cycle, so the
// near-null directions of Q - sigma that E approximates (the targets of the
// shifted inversions, including clustered ones) are handled in FP64 by a
// second, global coarse space built from the eigenvector approximations.
// ---------------------------------------------------------------------------
struct Deflation {
  const c128 *E = nullptr;
  int n = 0;
  std::vector<cd> LU[kMaxRhs];       // LU factors of A - sigma_k G (row-major)
  std::vector<int> piv[kMaxRhs];
};

// LU with partial pivoting, in place (row-major n x n).
bool lu_factor(int n, std::vector<cd> &M, std::vector<int> &piv) {
  piv.resize(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(M[(size_t)k * n + k]);
    for (int i = k + 1; i < n; ++i)
      if (std::abs(M[(size_t)i * n + k]) > best) { best = std::abs(M[(size_t)i * n + k]); p = i; }
    piv[k] = p;
    if (best == 0.0) return false;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(M[(size_t)k * n + j], M[(size_t)p * n + j]);
    const cd d = M[(size_t)k * n + k];
    for (int i = k + 1; i < n; ++i) {
      const cd f = M[(size_t)i * n + k] / d;
      M[(size_t)i * n + k] = f;
      for (int j = k + 1; j < n; ++j) M[(size_t)i * n + j] -= f * M[(size_t)k * n + j];
    }
  }
  return true;
}

void lu_solve(int n, const std::vector<cd> &M, const std::vector<int> &piv, cd *b) {
  for (int k = 0; k < n; ++k) {
    std::swap(b[k], b[piv[k]]);
    for (int i = k + 1; i < n; ++i) b[i] -= M[(size_t)i * n + k] * b[k];
  }
  for (int i = n - 1; i >= 0; --i) {
    cd v = b[i];
    for (int j = i + 1; j < n; ++j) v -= M[(size_t)i * n + j] * b[j];
    b[i] = v / M[(size_t)i * n + i];
  }
}

// Room for kMaxRhs FP64 fields outside the solves: the outer FGMRES basis
// when it is idle and large enough, else a buffer of its own.
c128 *idle_fields(lq_ctx *c) {
  const size_t need = (size_t)kMaxRhs * 12 * c->g.V;
  if (c->fine_kw.V.p && c->fine_kw.V.n >= need) return c->fine_kw.V.p;
  return c->defl_tmp.get(need);
}

// A = E^dag Q E and G = E^dag E for the n fields E (blocked layout, FP64).
void projected_operator(lq_ctx *c, const c128 *E, int n, std::vector<cd> &A, std::vector<cd> &G) {
  const long long V12 = 12LL * c->g.V;
  c128 *QE = idle_fields(c);
  A.assign((size_t)n * n, cd(0));
  G.assign((size_t)n * n, cd(0));
  Shifts z = shifts_of(nullptr, 0);
  for (int j0 = 0; j0 < n; j0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, n - j0);
    launch_wilson<double>(c->g, c->U64.p, E + j0 * V12, QE, nullptr, c->m0, z, nk, W_QSHIFT, c->st, clov_blk(c));
    auto a = gram(c, n, E, V12, nk, QE, V12, V12);
    auto g = gram(c, n, E, V12, nk, E + j0 * V12, V12, V12);
    for (int i = 0; i < n; ++i)
      for (int k = 0; k < nk; ++k) {
        A[(size_t)i * n + j0 + k] = a[(size_t)i * nk + k];
        G[(size_t)i * n + j0 + k] = g[(size_t)i * nk + k];
      }
  }
}

// After the fields E[ids[q]] were replaced by X[q] (q < nk, already copied into
// E), update their columns of A = E^dag Q E and G = E^dag E, and their rows by
// Hermiticity; the other entries do not change.
void update_projected(lq_ctx *c, const c128 *E, int n, const std::vector<int> &ids, const c128 *X,
                      std::vector<cd> &A, std::vector<cd> &G) {
  const long long V12 = 12LL * c->g.V;
  const int nk = (int)ids.size();
  c128 *QX = idle_fields(c);
  launch_wilson<double>(c->g, c->U64.p, X, QX, nullptr, c->m0, shifts_of(nullptr, 0), nk, W_QSHIFT, c->st,
                        clov_blk(c));
  auto a = gram(c, n, E, V12, nk, QX, V12, V12);
  auto g = gram(c, n, E, V12, nk, X, V12, V12);
  for (int q = 0; q < nk; ++q) {
    const int i = ids[q];
    for (int j = 0; j < n; ++j) {
      A[(size_t)j * n + i] = a[(size_t)j * nk + q];
      A[(size_t)i * n + j] = std::conj(a[(size_t)j * nk + q]);
      G[(size_t)j * n + i] = g[(size_t)j * nk + q];
      G[(size_t)i * n + j] = std::conj(g[(size_t)j * nk + q]);
    }
  }
}

// out = u + B_sigma(in - (Q - sigma) u) with u the Galerkin correction on span(E).
void deflated_precond(lq_ctx *c, const Deflation &D, const double *sig, const c128 *in, c128 *out, int nrhs) {
  const long long n = 12LL * c->g.V;
  auto cc = gram(c, D.n, D.E, n, nrhs, in, n, n);                    // [D.n][nrhs]
  std::vector<cd> Y(cc.size()), col(D.n);
  for (int k = 0; k < nrhs; ++k) {
    for (int i = 0; i < D.n; ++i) col[i] = cc[(size_t)i * nrhs + k];
    lu_solve(D.n, D.LU[k], D.piv[k], col.data());
    for (int i = 0; i < D.n; ++i) Y[(size_t)i * nrhs + k] = col[i];
  }
  c128 *U = c->defl_u.get((size_t)kMaxRhs * n), *R = c->defl_r.get((size_t)kMaxRhs * n);
  combine(c, D.n, D.E, n, nrhs, Y, 1.0, U, n, n, false);
  launch_wilson<double>(c->g, c->U64.p, U, R, in, c->m0, shifts_of(sig, nrhs), nrhs, W_RESID, c->st, clov_blk(c));
  precond64(c, sig, R, out, nrhs);
  launch_multi_axpy<double>(1, U, 0, n, c->plus_one.p, out, n, n, nrhs, 1.0, c->st);
}

void deflation_factor(Deflation &D, const std::vector<cd> &A, const std::vector<cd> &G, const double *sig,
                      int nrhs) {
  const int n = D.n;
  for (int k = 0; k < nrhs; ++k) {
    D.LU[k].resize((size_t)n * n);
    for (size_t e = 0; e < (size_t)n * n; ++e) D.LU[k][e] = A[e] - sig[k] * G[e];
    if (!lu_factor(n, D.LU[k], D.piv[k])) fail(LQ_ERR_NUMERIC, "projected shifted matrix is singular");
  }
}

void check_ctx(lq_ctx *c) {
  if (!c) fail(LQ_ERR_ARG, "NULL context");
  LQ_HIP(hipSetDevice(c->dev));
}
void need_mg(lq_ctx *c) {
  check_ctx(c);
  if (!c->have) fail(LQ_ERR_STATE, "mg_setup has not been called");
}

int guard(lq_ctx *c, const std::function<int()> &f) {
  try {
    if (c) c->err.clear();
    return f();
  } catch (const ApiError &e) {
    if (c) c->err = e.msg;
    return e.code;
  } catch (const HipError &e) {
    if (c) c->err = std::string("HIP error ") + hipGetErrorString(e.err) + " in " + e.what + " (" + e.file + ":" +
                    std::to_string(e.line) + ")";
    return LQ_ERR_HIP;
  } catch (const std::exception &e) {
    if (c) c->err = e.what();
    return LQ_ERR_HIP;
  }
}

}  // namespace

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

int lq_params_default(lq_mg_params *p) {
  if (!p) return LQ_ERR_ARG;
  p->precision = LQ_PREC_MIXED;
  p->smoother = LQ_SMOOTH_SAP;
  p->pre = 0;
  p->post = 3;
  p->sap_mr = 4;
  p->gmres_smooth_m = 8;
  p->coarse_m = 40;
  p->coarse_restarts = 4;
  p->coarse_tol = 0.05;
  p->fgmres_m = 10;
  p->fgmres_restarts = 40;
  p->n_init = 2;
  p->n_setup = 4;
  p->rqi_block = 16;
  p->rqi_max_sweeps = 30;
  p->rqi_solve_tol = 1e-6;
  p->rayleigh_ritz = 1;
  p->rqi_guard = 2;
  p->rqi_solve_restarts = 1;
  p->rqi_deflate = 1;
  p->rqi_start_passes = 0;
  p->graphs = 0;       // measured: replay gains nothing over direct launches here
  p->coarse_bf16 = 0;
  p->coarse2_m = 40;
  p->coarse2_restarts = 2;
  p->coarse2_tol = 0.1;
  p->smooth1_m = 4;
  p->post1 = 1;
  p->rqi_stall_restarts = 0;
  p->rqi_stall_eps = 1e-4;
  return LQ_OK;
}

int lq_create(lq_ctx **out, const int dims[4], int t_bc, void *stream) {
  if (!out || !dims) return LQ_ERR_ARG;
  *out = nullptr;
  for (int m = 0; m < 4; ++m)
    if (dims[m] < 2) return LQ_ERR_ARG;
  if (t_bc != 1 && t_bc != -1) return LQ_ERR_ARG;
  long long V = (long long)dims[0] * dims[1] * dims[2] * dims[3];
  if (V * 12 > (1LL << 31) - 1) return LQ_ERR_ARG;
  lq_ctx *c = new lq_ctx();
  for (int m = 0; m < 4; ++m) c->L[m] = dims[m];
  c->tbc = t_bc;
  c->st = (hipStream_t)stream;
  c->gcan = make_geom(dims, dims, t_bc);
  if (hipGetDevice(&c->dev) != hipSuccess) { delete c; return LQ_ERR_HIP; }
  // the allocation-free entry point's scratch, once per device (set-up time);
  // a failure only disables that entry point (it then returns LQ_ERR_STATE)
  (void)resolve_scratch(c->dev);
  lq_params_default(&c->p);
  int rc = guard(c, [&] {
    std::vector<c128> m1(kMaxRhs, c128{-1.0, 0.0}), p1(kMaxRhs, c128{1.0, 0.0});
    LQ_HIP(hipMemcpy(c->minus_one.get(kMaxRhs), m1.data(), kMaxRhs * sizeof(c128), hipMemcpyHostToDevice));
    LQ_HIP(hipMemcpy(c->plus_one.get(kMaxRhs), p1.data(), kMaxRhs * sizeof(c128), hipMemcpyHostToDevice));
    return LQ_OK;
  });
  if (rc != LQ_OK) { delete c; return rc; }
  *out = c;
  return LQ_OK;
}

int lq_destroy(lq_ctx *c) {
  if (!c) return LQ_ERR_ARG;
  (void)hipSetDevice(c->dev);
  (void)hipStreamSynchronize(c->st);
  delete c;
  return LQ_OK;
}

const char *lq_last_error(const lq_ctx *c) { return c ? c->err.c_str() : "NULL context"; }

int lq_clover(lq_ctx *c, const lq_c128 *U, double csw) {
  return guard(c, [&] {
    check_ctx(c);
    if ((!U && csw != 0) || !std::isfinite(csw)) fail(LQ_ERR_ARG, "lq_clover: NULL links or c_sw not finite");
    // a hierarchy built with the previous operator no longer matches it
    c->have = false;
    c->csw = csw;
    if (csw == 0) return LQ_OK;
    const long long CV = (long long)kCloverRows * c->gcan.V;
    launch_clover_build(c->gcan, (const c128 *)U, csw, c->clov_can.get(CV), c->st);
    launch_convert<float, double>(c->clov_can.p, c->clov_can32.get(CV), CV, c->st);
    sync(c);
    return LQ_OK;
  });
}

int q_apply(lq_ctx *c, const lq_c128 *U, double m0, const lq_c128 *x, lq_c128 *y, int n_rhs) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !x || !y || n_rhs < 1) fail(LQ_ERR_ARG, "q_apply: NULL pointer or n_rhs < 1");
    Shifts S = shifts_of(nullptr, 0);
    const long long L = 12LL * c->gcan.V;
    for (int k0 = 0; k0 < n_rhs; k0 += kMaxRhs) {
      const int nk = std::min(kMaxRhs, n_rhs - k0);
      launch_wilson<double>(c->gcan, (const c128 *)U, (const c128 *)x + k0 * L, (c128 *)y + k0 * L, nullptr, m0, S,
                            nk, W_QSHIFT, c->st, clov_can(c));
    }
    return LQ_OK;
  });
}

int q_apply_c64(lq_ctx *c, const lq_c64 *U, double m0, const lq_c64 *x, lq_c64 *y, int n_rhs) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !x || !y || n_rhs < 1) fail(LQ_ERR_ARG, "q_apply_c64: NULL pointer or n_rhs < 1");
    Shifts S = shifts_of(nullptr, 0);
    const long long L = 12LL * c->gcan.V;
    for (int k0 = 0; k0 < n_rhs; k0 += kMaxRhs) {
      const int nk = std::min(kMaxRhs, n_rhs - k0);
      launch_wilson<float>(c->gcan, (const c64 *)U, (const c64 *)x + k0 * L, (c64 *)y + k0 * L, nullptr, m0, S, nk,
                           W_QSHIFT, c->st, clov_can32(c));
    }
    return LQ_OK;
  });
}

int mg_setup(lq_ctx *c, const lq_c128 *U, double m0, int n_levels, const int n_tvs[], const int aggs[][4],
             const lq_c128 *tv0, const lq_mg_params *prm) {
  return guard(c, [&] {
    check_ctx(c);
    c->have = false;                     // a failed setup leaves no usable hierarchy
    // graphs captured for the previous hierarchy refer to its buffers and shapes
    drop_graphs(c);
    if (!U || !aggs || !n_tvs || !tv0) fail(LQ_ERR_ARG, "mg_setup: NULL pointer");
    if (n_levels != 2 && n_levels != 3) fail(LQ_ERR_ARG, "mg_setup: n_levels must be 2 or 3");
    const int *agg = aggs[0];
    const int n_tv = n_tvs[0];
    int bvol = 1;
    for (int m = 0; m < 4; ++m) {
      if (agg[m] < 1 || c->L[m] % agg[m]) fail(LQ_ERR_ARG, "aggregate extent does not divide the lattice");
      const int nb = c->L[m] / agg[m];
      if (nb != 1 && nb % 2) fail(LQ_ERR_ARG, "need 1 or an even number of aggregates per direction");
      bvol *= agg[m];
    }
    if (bvol > 256) fail(LQ_ERR_ARG, "aggregates hold at most 256 sites");
    if (n_tv < 1 || n_tv > 32 || n_tv > 6 * bvol) fail(LQ_ERR_ARG, "need 1 <= n_tv <= min(32, 6*|aggregate|)");
    lq_mg_params p;
    lq_params_default(&p);
    if (prm) p = *prm;
    if (p.smoother != LQ_SMOOTH_SAP) fail(LQ_ERR_ARG, "only the SAP smoother is implemented on the device");
    if (p.precision != LQ_PREC_FP64 && p.precision != LQ_PREC_MIXED) fail(LQ_ERR_ARG, "bad precision");
    if (p.rqi_block < 1 || p.rqi_block > kMaxRhs) fail(LQ_ERR_ARG, "rqi_block must be in 1..16");
    if (p.rqi_guard < 0) fail(LQ_ERR_ARG, "rqi_guard must be >= 0");
    if (p.rqi_start_passes < 0) fail(LQ_ERR_ARG, "rqi_start_passes must be >= 0");
    if (p.graphs != 0 && p.graphs != 1) fail(LQ_ERR_ARG, "graphs must be 0 or 1");
    if (p.coarse_bf16 != 0 && p.coarse_bf16 != 1) fail(LQ_ERR_ARG, "coarse_bf16 must be 0 or 1");
    if (p.coarse_bf16 && p.precision != LQ_PREC_MIXED) fail(LQ_ERR_ARG, "coarse_bf16 needs LQ_PREC_MIXED");
    if (p.rqi_stall_restarts < 0 || !(p.rqi_stall_eps >= 0)) fail(LQ_ERR_ARG, "mg_setup: bad straggler parameters");
    if (p.coarse_m < 1 || p.fgmres_m < 1 || p.sap_mr < 0 || p.post < 0 || p.pre < 0)
      fail(LQ_ERR_ARG, "bad iteration parameters");
    c->p = p;
    c->m0 = m0;
    c->Nv = n_tv;
    for (int m = 0; m < 4; ++m) c->agg[m] = agg[m];
    c->g = make_geom(c->L, agg, c->tbc);
    for (int m = 0; m < 4; ++m) c->cg.nb[m] = c->g.nb[m];
    c->cg.nA = c->g.nblk;
    c->cg.n2 = 2 * n_tv;
    c->n_levels = n_levels;
    if (n_levels == 3) {
      const int *agg2 = aggs[1];
      const int nv2 = n_tvs[1];
      if (p.coarse2_m < 1 || p.coarse2_restarts < 0 || p.smooth1_m < 1 || p.post1 < 0)
        fail(LQ_ERR_ARG, "bad level-2 iteration parameters");
      Level2Geom &l2 = c->l2g;
      l2.bvol2 = 1;
      l2.nA2 = 1;
      for (int m = 0; m < 4; ++m) {
        if (agg2[m] < 1 || c->cg.nb[m] % agg2[m]) fail(LQ_ERR_ARG, "level-2 aggregate extent does not divide the "
                                                                   "lattice of aggregates");
        l2.nb1[m] = c->cg.nb[m];
        l2.b2[m] = agg2[m];
        l2.nb2[m] = c->cg.nb[m] / agg2[m];
        l2.bvol2 *= agg2[m];
        l2.nA2 *= l2.nb2[m];
        c->agg2[m] = agg2[m];
        c->cg2.nb[m] = l2.nb2[m];
      }
      if (nv2 < 1 || nv2 > 32 || nv2 > n_tv) fail(LQ_ERR_ARG, "need 1 <= n_tv[1] <= min(32, n_tv[0])");
      l2.nA1 = c->cg.nA;
      l2.Nv1 = n_tv;
      l2.Nv2 = nv2;
      c->Nv2 = nv2;
      c->cg2.nA = l2.nA2;
      c->cg2.n2 = 2 * nv2;
    } else {
      c->Nv2 = 0;
    }
    const long long V = c->g.V, V12 = 12LL * V;
    // links
    launch_pack_links<double>(c->g, (const c128 *)U, c->U64.get(36 * V), c->st);
    if (p.precision == LQ_PREC_FP64) copy<double>(c, c->d64.U.get(36 * V), c->U64.p, 36 * V);
    else launch_pack_links<float>(c->g, (const c128 *)U, c->d32.U.get(36 * V), c->st);
    // the clover term of lq_clover in the blocked layout (rows as 4 fields of 12)
    if (c->csw != 0) {
      const long long CV = (long long)kCloverRows * V;
      launch_permute<double>(c->g, c->clov_can.p, c->clov64.get(CV), kCloverRows / 12, true, c->st);
      if (p.precision == LQ_PREC_FP64) copy<double>(c, c->d64.C.get(CV), c->clov64.p, CV);
      else launch_convert<float, double>(c->clov64.p, c->d32.C.get(CV), CV, c->st);
    }
    // red / black block lists
    std::vector<int> lists[2];
    for (int A = 0; A < c->g.nblk; ++A) {
      int r = A, s = 0;
      for (int m = 0; m < 3; ++m) { s += r % c->g.nb[m]; r /= c->g.nb[m]; }
      s += r;
      lists[s & 1].push_back(A);
    }
    for (int col = 0; col < 2; ++col) {
      c->nblocks[col] = (int)lists[col].size();
      int *d = c->blocks[col].get(std::max<size_t>(1, lists[col].size()));
      if (!lists[col].empty())
        LQ_HIP(hipMemcpyAsync(d, lists[col].data(), lists[col].size() * sizeof(int), hipMemcpyHostToDevice, c->st));
    }
    // test vectors
    c128 *W = c->W.get((size_t)n_tv * V12);
    launch_permute<double>(c->g, (const c128 *)tv0, W, n_tv, true, c->st);
    c128 *tmp = c->tmpA.get((size_t)kMaxRhs * V12);
    std::vector<double> zs(kMaxRhs, 0.0);
    for (int it = 0; it < p.n_init; ++it)
      for (int k0 = 0; k0 < n_tv; k0 += kMaxRhs) {
        const int nk = std::min(kMaxRhs, n_tv - k0);
        smooth64(c, zs.data(), W + k0 * V12, tmp, nk, std::max(p.post, 1));
        copy<double>(c, W + k0 * V12, tmp, (size_t)nk * V12);
      }
    orthonormalise(c, W, n_tv);
    rebuild(c, fields_of(c, W, n_tv));   // dependent start vectors are an error
    for (int it = 0; it < p.n_setup; ++it) {
      for (int k0 = 0; k0 < n_tv; k0 += kMaxRhs) {
        const int nk = std::min(kMaxRhs, n_tv - k0);
        precond64(c, zs.data(), W + k0 * V12, tmp, nk);
        copy<double>(c, W + k0 * V12, tmp, (size_t)nk * V12);
      }
      orthonormalise(c, W, n_tv);
      // vectors the multigrid iteration made locally dependent (a near-null
      // space thinner than Nv on some aggregate) leave those blocks of P as
      // they were
      rebuild(c, fields_of(c, W, n_tv), true);
      if (verbose()) {
        size_t fr = 0, tot = 0;
        (void)hipMemGetInfo(&fr, &tot);
        std::fprintf(stderr, "[lqmg] setup pass %d/%d done, coarse its so far %d, device memory free %zu MiB\n",
                     it + 1, p.n_setup, c->coarse_iters, fr >> 20);
        std::fflush(stderr);
      }
    }
    sync(c);
    c->have = true;                      // only a setup that completed is usable
    return LQ_OK;
  });
}

int mg_solve_shifted(lq_ctx *c, int n_rhs, const double *sigma, const lq_c128 *rhs, lq_c128 *x, double tol,
                     lq_solve_stats *st) {
  return guard(c, [&] {
    need_mg(c);
    if (n_rhs < 1 || n_rhs > kMaxRhs || !sigma || !rhs || !x || !(tol > 0))
      fail(LQ_ERR_ARG, "mg_solve_shifted: bad arguments");
    const long long V12 = 12LL * c->g.V;
    c128 *b = c->tmpA.get((size_t)kMaxRhs * V12);
    c128 *xb = c->tmpB.get((size_t)kMaxRhs * V12);
    launch_permute<double>(c->g, (const c128 *)rhs, b, n_rhs, true, c->st);
    int its[kMaxRhs];
    double rr[kMaxRhs];
    c->coarse_iters = 0;
    bool ok = solve_shifted(c, n_rhs, sigma, b, xb, tol, its, rr, c->p.fgmres_restarts);
    launch_permute<double>(c->g, xb, (c128 *)x, n_rhs, false, c->st);
    sync(c);
    if (st) {
      std::memset(st, 0, sizeof(*st));
      for (int k = 0; k < n_rhs; ++k) { st->iters[k] = its[k]; st->relres[k] = rr[k]; }
      st->coarse_iters = c->coarse_iters;
    }
    return ok ? LQ_OK : LQ_WARN_NOCONV;
  });
}

int rqi_lowmodes(lq_ctx *c, int n_eig, double tol, double *lambda, lq_c128 *Vout, double *resid, const lq_c128 *V0,
                 int n_v0, lq_rqi_stats *stats) {
  return guard(c, [&] {
    need_mg(c);
    if (n_eig < 1 || !(tol > 0) || !lambda || !Vout || !resid) fail(LQ_ERR_ARG, "rqi_lowmodes: bad arguments");
    const int Nv = c->Nv;
    const long long V12 = 12LL * c->g.V;
    const int nw = n_eig + std::max(0, c->p.rqi_guard);        // working vectors
    const int n_tv_used = std::min(Nv, nw);
    if (n_v0 == nw) {
      if (!V0) fail(LQ_ERR_ARG, "V0 is NULL");
    } else if (n_v0 != nw - n_tv_used) {
      fail(LQ_ERR_ARG, "n_v0 must be n_work - min(Nv, n_work) or n_work (n_work = n_eig + rqi_guard)");
    } else if (n_v0 > 0 && !V0) {
      fail(LQ_ERR_ARG, "V0 is NULL");
    }
    lq_rqi_stats S;
    std::memset(&S, 0, sizeof(S));
    c128 *E = c->eig.get((size_t)nw * V12);
    if (n_v0 == nw) {
      launch_permute<double>(c->g, (const c128 *)V0, E, nw, true, c->st);
    } else {
      copy<double>(c, E, c->W.p, (size_t)n_tv_used * V12);
      if (n_v0 > 0) launch_permute<double>(c->g, (const c128 *)V0, E + n_tv_used * V12, n_v0, true, c->st);
    }
    // Alg. 1 starts from orthonormal vectors (also before start passes: the
    // first multigrid pass then acts on an orthonormal set)
    orthonormalise(c, E, nw);
    std::vector<double> lam(nw, 0.0), eps(nw, 1.0);

    // P from the current approximations (Alg. 1 puts each new iterate into
    // the interpolation).  With
    // more vectors than Nv it takes the Nv whose lambda lies nearest to one of
    // the shifts about to be solved for (ties: lower index), so that the
    // coarse space holds the near-null vectors of those Q - sigma.
    auto rebuild_from = [&](const std::vector<double> &shifts) {
      double t0 = now();
      std::vector<int> idx;
      if (nw <= Nv) {
        for (int i = 0; i < nw; ++i) idx.push_back(i);
      } else {
        std::vector<double> dist(nw);
        for (int i = 0; i < nw; ++i) {
          dist[i] = 1e300;
          for (double s : shifts) dist[i] = std::min(dist[i], std::fabs(lam[i] - s));
        }
        std::vector<int> o(nw);
        for (int i = 0; i < nw; ++i) o[i] = i;
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return dist[a] < dist[b]; });
        idx.assign(o.begin(), o.begin() + Nv);
        std::sort(idx.begin(), idx.end());
      }
      std::vector<const c128 *> src(Nv);
      for (size_t q = 0; q < idx.size(); ++q) src[q] = E + idx[q] * V12;
      for (int q = (int)idx.size(); q < Nv; ++q) src[q] = c->W.p + q * V12;
      // approximations that are dependent on an aggregate (exactly degenerate
      // smooth modes) leave that aggregate's columns of P as they were
      if (rebuild(c, src, true)) S.p_rebuilds++;
      S.t_rebuild += now() - t0;
    };
    // the n_eig vectors with smallest |lambda| have converged
    auto wanted_done = [&]() {
      std::vector<int> o(nw);
      for (int i = 0; i < nw; ++i) o[i] = i;
      std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return std::fabs(lam[a]) < std::fabs(lam[b]); });
      for (int q = 0; q < n_eig; ++q)
        if (!(eps[o[q]] <= tol)) return false;
      return true;
    };
    rebuild_from({0.0});
    c128 *X = c->tmpB.get((size_t)kMaxRhs * V12);
    c128 *B = c->tmpA.get((size_t)kMaxRhs * V12);
    const int nb = c->p.rqi_block;
    // the FGMRES basis takes its solve shape now: Rayleigh-Ritz borrows it as
    // scratch, and sizing it for that first would leave no room for the solves
    {
      const size_t blk = (size_t)std::min(nb, nw);
      c->fine_kw.V.get((size_t)(c->p.fgmres_m + 1) * blk * V12);
      c->fine_kw.Z.get((size_t)c->p.fgmres_m * blk * V12);
    }
    // lambda_i and eps_i = ||Q v_i - lambda_i v_i|| for the listed vectors
    auto rq_resid = [&](const std::vector<int> &ids) {
      for (size_t q0 = 0; q0 < ids.size(); q0 += kMaxRhs) {
        const int nk = (int)std::min<size_t>(kMaxRhs, ids.size() - q0);
        for (int q = 0; q < nk; ++q) copy<double>(c, B + q * V12, E + ids[q0 + q] * V12, V12);
        Shifts z = shifts_of(nullptr, 0);
        launch_wilson<double>(c->g, c->U64.p, B, X, nullptr, c->m0, z, nk, W_QSHIFT, c->st, clov_blk(c));
        // all nk pairs at once: lambda_q = <v_q, Q v_q>, X_q <- Q v_q - lambda_q v_q, eps_q = |X_q|
        auto d = dots<double>(c, 1, B, 0, V12, X, V12, V12, nk);
        std::vector<cd> lq(nk);
        for (int q = 0; q < nk; ++q) {
          lam[ids[q0 + q]] = d[q].real();
          lq[q] = cd(d[q].real());
        }
        axpys<double>(c, 1, B, 0, V12, lq, X, V12, V12, nk, -1.0);
        auto nr = norms<double>(c, X, V12, nk);
        for (int q = 0; q < nk; ++q) eps[ids[q0 + q]] = nr[q];
      }
    };
    // Rayleigh-Ritz on E[L..nw) (orthonormal, orthogonal to E[0..L)), then
    // lambda and eps of those vectors.  The FGMRES basis vectors (V, then Z)
    // are idle here and hold the rotated vectors; only if they are too few is
    // more memory taken.
    auto rr_tail = [&](int L) {
      std::vector<c128 *> spill;
      const size_t nV = c->fine_kw.V.n / V12, nZ = c->fine_kw.Z.n / V12;
      if (nV + nZ >= (size_t)(nw - L)) {
        for (int j = 0; j < nw - L; ++j)
          spill.push_back((size_t)j < nV ? c->fine_kw.V.p + j * V12 : c->fine_kw.Z.p + (j - nV) * V12);
      } else {
        c128 *sp = c->fine_kw.V.get((size_t)(nw - L) * V12);
        for (int j = 0; j < nw - L; ++j) spill.push_back(sp + j * V12);
      }
      rayleigh_ritz_tail(c, E, nw, L, lam, spill);
      std::vector<int> U;
      for (int i = L; i < nw; ++i) U.push_back(i);
      rq_resid(U);
    };
    // Start passes: the setup's multigrid iteration (sec. 2.1) over every
    // start vector, v <- M_0 v with the sigma = 0 preconditioner, keeping the
    // set orthonormal; a Rayleigh-Ritz step then gives lambda_i and eps_i, and
    // P is rebuilt from the vectors with the smallest |lambda|.
    for (int pass = 0; pass < c->p.rqi_start_passes; ++pass) {
      double t0 = now();
      std::vector<double> zs(kMaxRhs, 0.0);
      for (int k0 = 0; k0 < nw; k0 += kMaxRhs) {
        const int nk = std::min(kMaxRhs, nw - k0);
        precond64(c, zs.data(), E + k0 * V12, X, nk);
        copy<double>(c, E + k0 * V12, X, (size_t)nk * V12);
      }
      S.t_solve += now() - t0;
      t0 = now();
      if (c->p.rayleigh_ritz) {
        rr_tail(0);                 // generalised Rayleigh-Ritz: its Ritz vectors are orthonormal
      } else {
        orthonormalise(c, E, nw);
        rq_resid([&] { std::vector<int> a(nw); for (int i = 0; i < nw; ++i) a[i] = i; return a; }());
      }
      S.t_rq += now() - t0;
      rebuild_from({0.0});
      if (verbose()) {
        double emax = 0;
        for (int i = 0; i < nw; ++i) emax = std::max(emax, eps[i]);
        std::fprintf(stderr, "[lqmg] rqi start pass %d/%d: max eps %.3e\n", pass + 1, c->p.rqi_start_passes, emax);
        std::fflush(stderr);
      }
    }
    // A = E^dag Q E and G = E^dag E for the Galerkin correction, kept up to date
    // column by column as block members change; recomputed after rotations
    std::vector<cd> Aop, Gop;
    bool ag_valid = false;
    bool done = false;
    // residuals at the start of the previous sweep, by slot (stragglers)
    std::vector<double> eps_prev(nw, std::numeric_limits<double>::infinity());
    while (!done && S.sweeps < c->p.rqi_max_sweeps) {
      // unconverged vectors; stragglers (below rqi_stall_eps, less than halved
      // over the last sweep) go last, in blocks of their own with more restarts
      std::vector<int> todo, slow;
      for (int i = 0; i < nw; ++i) {
        if (!(eps[i] > tol)) continue;
        const bool stalled = c->p.rqi_stall_restarts > 0 && eps[i] < c->p.rqi_stall_eps && eps[i] > 0.5 * eps_prev[i];
        (stalled ? slow : todo).push_back(i);
      }
      const size_t n_fast = todo.size();
      todo.insert(todo.end(), slow.begin(), slow.end());
      eps_prev = eps;
      if (todo.empty()) break;
      for (size_t q0 = 0, step = 0; q0 < todo.size(); q0 += step) {
        // blocks of nb, the last fast block cut short so no block mixes the two groups
        const int nk = (int)std::min<size_t>(nb, (q0 < n_fast ? n_fast : todo.size()) - q0);
        step = (size_t)nk;
        const bool boost = q0 >= n_fast;
        std::vector<double> sig(nk);
        for (int q = 0; q < nk; ++q) {
          const int i = todo[q0 + q];
          sig[q] = lam[i] * std::max(1.0 - eps[i], 0.0);        // damped shift (Alg. 1)
          copy<double>(c, B + q * V12, E + i * V12, V12);
        }
        if (nw > Nv) rebuild_from(sig);
        double t0 = now();
        Deflation D;
        if (c->p.rqi_deflate) {
          if (!ag_valid) {
            projected_operator(c, E, nw, Aop, Gop);
            ag_valid = true;
          }
          D.E = E;
          D.n = nw;
          deflation_factor(D, Aop, Gop, sig.data(), nk);
        }
        int its[kMaxRhs];
        double rr[kMaxRhs];
        solve_shifted(c, nk, sig.data(), B, X, c->p.rqi_solve_tol, its, rr,
                      c->p.rqi_solve_restarts + (boost ? c->p.rqi_stall_restarts : 0), c->p.rqi_deflate ? &D : nullptr);
        for (int q = 0; q < nk; ++q) S.fgmres_iters += its[q];
        S.solves += nk;
        S.t_solve += now() - t0;
        t0 = now();
        // Gram-Schmidt (twice): first against the vectors outside the block
        // that precede each member or are locked, all block members at once ...
        std::vector<char> inblk(nw, 0);
        for (int q = 0; q < nk; ++q) inblk[todo[q0 + q]] = 1;
        for (int pass = 0; pass < 2; ++pass) {
          auto h = gram(c, nw, E, V12, nk, X, V12, V12);                // h[j][q] = <E_j, X_q>
          for (int j = 0; j < nw; ++j)
            for (int q = 0; q < nk; ++q) {
              const int i = todo[q0 + q];
              const bool use = !inblk[j] && (j < i || eps[j] <= tol);
              if (!use) h[(size_t)j * nk + q] = 0;
            }
          combine(c, nw, E, V12, nk, h, -1.0, X, V12, V12, true);
        }
        // ... then among the block members in index order, normalising each.
        for (int q = 0; q < nk; ++q) {
          const int i = todo[q0 + q];
          c128 *x = X + q * V12;
          if (q > 0)
            for (int pass = 0; pass < 2; ++pass) {
              auto h = dots<double>(c, q, X, V12, 0, x, 0, V12, 1);
              axpys<double>(c, q, X, V12, 0, h, x, 0, V12, 1, -1.0);
            }
          auto nr = norms<double>(c, x, V12, 1);
          if (!(nr[0] > 0) || !std::isfinite(nr[0])) fail(LQ_ERR_NUMERIC, "RQI iterate collapsed");
          scale<double>(c, std::vector<cd>{cd(1.0 / nr[0])}, x, 0, x, 0, V12, 1, false);
          copy<double>(c, E + i * V12, x, V12);
        }
        if (c->p.rqi_deflate && ag_valid)
          update_projected(c, E, nw, std::vector<int>(todo.begin() + q0, todo.begin() + q0 + nk), X, Aop, Gop);
        S.t_ortho += now() - t0;
        if (nw <= Nv) rebuild_from(sig);       // P holds every vector: put the new ones in
        t0 = now();
        rq_resid(std::vector<int>(todo.begin() + q0, todo.begin() + q0 + nk));
        S.t_rq += now() - t0;
        if (verbose()) {
          int itmax = 0;
          double rmax = 0, rmin = 1e300;
          for (int q = 0; q < nk; ++q) {
            itmax = std::max(itmax, its[q]);
            rmax = std::max(rmax, rr[q]);
            rmin = std::min(rmin, rr[q]);
          }
          std::fprintf(stderr, "[lqmg]   sweep %d block at %zu: %d solves, max fgmres its %d, relres %.1e..%.1e, "
                       "coarse its %d\n", S.sweeps + 1, q0, nk, itmax, rmin, rmax, c->coarse_iters);
          std::fflush(stderr);
        }
      }
      S.sweeps++;
      if (c->p.rayleigh_ritz) {
        // Rayleigh-Ritz among the unconverged vectors, after orthonormalising
        // them against the locked (converged) ones; locked pairs stay as they are.
        // The converged vectors are first moved to the front slots.
        std::vector<int> order;
        for (int i = 0; i < nw; ++i)
          if (eps[i] <= tol) order.push_back(i);
        const int L = (int)order.size();
        for (int i = 0; i < nw; ++i)
          if (eps[i] > tol) order.push_back(i);
        if (nw - L > 1) {
          double t0 = now();
          permute_fields(c, E, order, c->tmpB.get((size_t)kMaxRhs * V12));
          std::vector<double> l2(nw), e2(nw);
          for (int p = 0; p < nw; ++p) { l2[p] = lam[order[p]]; e2[p] = eps[order[p]]; }
          lam = l2;
          eps = e2;
          rr_tail(L);
          ag_valid = false;
          S.t_rq += now() - t0;
          if (nw <= Nv) rebuild_from({0.0});
        }
      }
      done = wanted_done();
      if (verbose()) {
        int nconv = 0;
        double emax = 0;
        for (int i = 0; i < nw; ++i) {
          nconv += eps[i] <= tol;
          emax = std::max(emax, eps[i]);
        }
        // the n_eig wanted (smallest |lambda|): how many have converged, worst residual
        std::vector<int> o(nw);
        for (int i = 0; i < nw; ++i) o[i] = i;
        std::stable_sort(o.begin(), o.end(), [&](int a, int b) { return std::fabs(lam[a]) < std::fabs(lam[b]); });
        int wconv = 0;
        double wmax = 0;
        for (int q = 0; q < n_eig; ++q) {
          wconv += eps[o[q]] <= tol;
          wmax = std::max(wmax, eps[o[q]]);
        }
        std::fprintf(stderr, "[lqmg] rqi sweep %d: %d/%d converged (wanted %d/%d, max eps %.2e), max eps %.3e, "
                     "solves %d, fgmres its %d, t solve %.2fs ortho %.2fs rebuild %.2fs rq %.2fs\n", S.sweeps,
                     nconv, nw, wconv, n_eig, wmax, emax, S.solves, S.fgmres_iters, S.t_solve, S.t_ortho,
                     S.t_rebuild, S.t_rq);
        std::fflush(stderr);
      }
    }
    // output: the n_eig smallest |lambda|, sorted by (|lambda|, lambda)
    std::vector<int> o(nw);
    for (int i = 0; i < nw; ++i) o[i] = i;
    std::sort(o.begin(), o.end(), [&](int a, int b) {
      if (std::fabs(lam[a]) != std::fabs(lam[b])) return std::fabs(lam[a]) < std::fabs(lam[b]);
      return lam[a] < lam[b];
    });
    for (int q = 0; q < n_eig; ++q) {
      lambda[q] = lam[o[q]];
      resid[q] = eps[o[q]];
      launch_permute<double>(c->g, E + o[q] * V12, (c128 *)Vout + q * V12, 1, false, c->st);
    }
    sync(c);
    if (stats) *stats = S;
    return done ? LQ_OK : LQ_WARN_NOCONV;
  });
}

int lq_ptc_forward(lq_ctx *c, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out, const lq_c128 *W,
                   lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !phi || !W || !out || c_in < 1 || c_in > 64 || c_out < 1 || c_out > 64)
      fail(LQ_ERR_ARG, "lq_ptc_forward: NULL pointer or channel count outside 1..64");
    launch_ptc_forward(c->gcan, (const c128 *)U, c_in, (const c128 *)phi, c_out, (const c128 *)W, (c128 *)out,
                       c->st);
    return LQ_OK;
  });
}

int lq_ptc_forward_bf16(lq_ctx *c, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out, const lq_c128 *W,
                        lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !phi || !W || !out || c_in < 1 || c_in > 24 || c_out < 1 || c_out > 24)
      fail(LQ_ERR_ARG, "lq_ptc_forward_bf16: NULL pointer or channel count outside 1..24");
    unsigned *sc = c->ptc_bf16.get(ptc_bf16_scratch_words(c->gcan.V, c_in, c_out));
    launch_ptc_forward_bf16(c->gcan, (const c128 *)U, c_in, (const c128 *)phi, c_out, (const c128 *)W,
                            (c128 *)out, sc, c->st);
    return LQ_OK;
  });
}

int lq_ptc_backward(lq_ctx *c, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out, const lq_c128 *W,
                    const lq_c128 *g_out, lq_c128 *g_in, lq_c128 *g_W) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !phi || !W || !g_out || c_in < 1 || c_in > 64 || c_out < 1 || c_out > 64)
      fail(LQ_ERR_ARG, "lq_ptc_backward: NULL pointer or channel count outside 1..64");
    launch_ptc_backward(c->gcan, (const c128 *)U, c_in, (const c128 *)phi, c_out, (const c128 *)W,
                        (const c128 *)g_out, (c128 *)g_in, (c128 *)g_W, c->st);
    return LQ_OK;
  });
}

int lq_ptc_backward_bf16(lq_ctx *c, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out, const lq_c128 *W,
                         const lq_c128 *g_out, lq_c128 *g_in, lq_c128 *g_W) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !phi || !W || !g_out || c_in < 1 || c_in > 24 || c_out < 1 || c_out > 24)
      fail(LQ_ERR_ARG, "lq_ptc_backward_bf16: NULL pointer or channel count outside 1..24");
    if (!g_in && !g_W) return LQ_OK;
    unsigned *sc = c->ptc_bf16.get(ptc_bf16_backward_scratch_words(c->gcan.V, c_in, c_out));
    launch_ptc_backward_bf16(c->gcan, (const c128 *)U, c_in, (const c128 *)phi, c_out, (const c128 *)W,
                             (const c128 *)g_out, (c128 *)g_in, (c128 *)g_W, sc, c->st);
    return LQ_OK;
  });
}

int lq_mod_relu(lq_ctx *c, int channels, const lq_c128 *phi, const double *b, lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (!phi || !b || !out || channels < 1 || channels > 64)
      fail(LQ_ERR_ARG, "lq_mod_relu: NULL pointer or channel count outside 1..64");
    launch_mod_relu(c->gcan.V, channels, (const c128 *)phi, b, (c128 *)out, c->st);
    return LQ_OK;
  });
}

int lq_mod_relu_backward(lq_ctx *c, int channels, const lq_c128 *phi, const double *b, const lq_c128 *g_out,
                         lq_c128 *g_phi, double *g_b) {
  return guard(c, [&] {
    check_ctx(c);
    if (!phi || !b || !g_out || !g_phi || !g_b || channels < 1 || channels > 64)
      fail(LQ_ERR_ARG, "lq_mod_relu_backward: NULL pointer or channel count outside 1..64");
    double *scr = c->net_scratch.get((size_t)channels * c->gcan.V);
    launch_mod_relu_backward(c->gcan.V, channels, (const c128 *)phi, b, (const c128 *)g_out, (c128 *)g_phi, g_b, scr,
                             c->st);
    return LQ_OK;
  });
}

int lq_proj_loss(lq_ctx *c, const int agg[4], int n_out, const lq_c128 *X, int K, const lq_c128 *u, double *loss,
                 lq_c128 *g_X) {
  return guard(c, [&] {
    check_ctx(c);
    if (!agg || !X || !u || !loss || n_out < 1 || n_out > 32 || K < 1 || K > 32)
      fail(LQ_ERR_ARG, "lq_proj_loss: NULL pointer or n_out / K outside 1..32");
    int bvol = 1, nblk = 1;
    for (int m = 0; m < 4; ++m) {
      if (agg[m] < 1 || c->L[m] % agg[m]) fail(LQ_ERR_ARG, "lq_proj_loss: aggregate extent does not divide the lattice");
      bvol *= agg[m];
      nblk *= c->L[m] / agg[m];
    }
    if (n_out > 6 * bvol) fail(LQ_ERR_ARG, "lq_proj_loss: more outputs than rows of an aggregate half");
    double *part = c->net_scratch.get((size_t)2 * nblk + 1);
    int *st = c->status.get(1);
    LQ_HIP(hipMemsetAsync(st, 0, sizeof(int), c->st));
    launch_proj_loss(c->L, agg, n_out, (const c128 *)X, K, (const c128 *)u, part, part + 2 * nblk, (c128 *)g_X, st,
                     c->st);
    double h_loss = 0;
    int h_st = 0;
    LQ_HIP(hipMemcpyAsync(&h_loss, part + 2 * nblk, sizeof(double), hipMemcpyDeviceToHost, c->st));
    LQ_HIP(hipMemcpyAsync(&h_st, st, sizeof(int), hipMemcpyDeviceToHost, c->st));
    sync(c);
    if (h_st) fail(LQ_ERR_NUMERIC, "lq_proj_loss: outputs linearly dependent on an aggregate half");
    *loss = h_loss;
    return LQ_OK;
  });
}

int lq_adam_step(lq_ctx *c, long long n, double *p, const double *g, double *m, double *v, double lr, double beta1,
                 double beta2, double eps, int t) {
  return guard(c, [&] {
    check_ctx(c);
    if (n < 0 || (n > 0 && (!p || !g || !m || !v)) || t < 1 || !(beta1 >= 0 && beta1 < 1) ||
        !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
      fail(LQ_ERR_ARG, "lq_adam_step: bad arguments");
    launch_adam(n, p, g, m, v, lr, beta1, beta2, eps, t, c->st);
    return LQ_OK;
  });
}

int lq_coarse_variant(int v) { return coarse_force_variant(v) == 0 ? LQ_OK : LQ_ERR_ARG; }

int lq_herm_eigh(int n, const lq_c128 *A, double *w, lq_c128 *V) {
  if (n < 1 || !A || !w || !V) return LQ_ERR_ARG;
  try {
    std::vector<cd> M((size_t)n * n), Z;
    std::memcpy(M.data(), A, M.size() * sizeof(cd));
    for (int i = 0; i < n; ++i)                       // use the Hermitian part
      for (int j = i; j < n; ++j) {
        const cd h = 0.5 * (M[(size_t)i * n + j] + std::conj(M[(size_t)j * n + i]));
        M[(size_t)i * n + j] = h;
        M[(size_t)j * n + i] = std::conj(h);
      }
    herm_eigh(n, M, Z);
    std::vector<int> o(n);
    for (int i = 0; i < n; ++i) o[i] = i;
    std::stable_sort(o.begin(), o.end(),
                     [&](int a, int b) { return M[(size_t)a * n + a].real() < M[(size_t)b * n + b].real(); });
    for (int j = 0; j < n; ++j) {
      w[j] = M[(size_t)o[j] * n + o[j]].real();
      for (int i = 0; i < n; ++i) {
        const cd z = Z[(size_t)i * n + o[j]];
        V[(size_t)i * n + j] = lq_c128{z.real(), z.imag()};
      }
    }
  } catch (...) {
    return LQ_ERR_NUMERIC;
  }
  return LQ_OK;
}

int lq_inner_products(lq_ctx *c, int nb, const lq_c128 *E, int nw, const lq_c128 *W, long long n, lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (nb < 1 || nb > 192 || nw < 1 || nw > 16 || n < 1 || !E || !W || !out)
      fail(LQ_ERR_ARG, "lq_inner_products: bad arguments");
    auto g = gram(c, nb, (const c128 *)E, n, nw, (const c128 *)W, n, n);
    std::memcpy(out, g.data(), g.size() * sizeof(cd));
    return LQ_OK;
  });
}

int lq_inner_products_noalloc(lq_ctx *c, int nb, const lq_c128 *E, int nw, const lq_c128 *W, long long n,
                              lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (nb < 1 || nb > 192 || nw < 1 || nw > 16 || n < 1 || !E || !W || !out)
      fail(LQ_ERR_ARG, "lq_inner_products_noalloc: need 1 <= nb <= 192, 1 <= nw <= 16, n >= 1, non-NULL pointers");
    unsigned char *base = static_cast<unsigned char *>(scratch_on(c->dev));
    if (!base) fail(LQ_ERR_STATE, "lq_inner_products_noalloc: no scratch address for this device");
    // results first, then as many element chunks of partial sums as fit
    c128 *dout = reinterpret_cast<c128 *>(base);
    c128 *part = reinterpret_cast<c128 *>(base + kNoAllocOutBytes);
    const long long max_chunks =
        (long long)((kNoAllocBytes - kNoAllocOutBytes) / (gram_chunk_elems(nb) * sizeof(c128)));
    launch_gram(nb, (const c128 *)E, n, nw, (const c128 *)W, n, n, dout, part, c->st, max_chunks);
    LQ_HIP(hipMemcpyAsync(out, dout, (size_t)nb * nw * sizeof(c128), hipMemcpyDeviceToHost, c->st));
    sync(c);
    return LQ_OK;
  });
}

}  // extern "C"

namespace {

// Approximate low-mode averaging (sec. 3.2-3.3): the kept approximations
// (eps_i <= cutoff |lambda_i|) copied to lma_V, and A = V^dag Q V with its LU.
struct LmaLow {
  int n = 0;
  std::vector<cd> A, LU;
  std::vector<int> piv;
};

LmaLow lma_prepare(lq_ctx *c, const c128 *U, double m0, int n, const c128 *V, const double *lam, const double *eps,
                   double cutoff) {
  const long long V12 = 12LL * c->gcan.V;
  std::vector<int> keep;
  for (int i = 0; i < n; ++i)
    if (eps[i] <= cutoff * std::fabs(lam[i])) keep.push_back(i);
  LmaLow L;
  L.n = (int)keep.size();
  if (L.n == 0) return L;
  if (L.n > 192) fail(LQ_ERR_ARG, "at most 192 approximations are kept");
  c128 *Vk = c->lma_V.get((size_t)L.n * V12);
  for (int q = 0; q < L.n; ++q) copy<double>(c, Vk + q * V12, V + keep[q] * V12, V12);
  c128 *QV = c->lma_W.get((size_t)kMaxRhs * V12);
  L.A.assign((size_t)L.n * L.n, cd(0));
  Shifts z = shifts_of(nullptr, 0);
  for (int j0 = 0; j0 < L.n; j0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, L.n - j0);
    launch_wilson<double>(c->gcan, U, Vk + j0 * V12, QV, nullptr, m0, z, nk, W_QSHIFT, c->st, clov_can(c));
    auto a = gram(c, L.n, Vk, V12, nk, QV, V12, V12);
    for (int i = 0; i < L.n; ++i)
      for (int k = 0; k < nk; ++k) L.A[(size_t)i * L.n + j0 + k] = a[(size_t)i * nk + k];
  }
  L.LU = L.A;
  if (!lu_factor(L.n, L.LU, L.piv)) fail(LQ_ERR_NUMERIC, "the projected matrix A is singular");
  return L;
}


// ---------------------------------------------------------------------------
// Restarted Lanczos on Q^2 (the Krylov comparison of sec. 2.2): the n_eig
// eigenvalues of Q of smallest modulus are the smallest of Q^2.  Each cycle
// extends the basis to n_kv vectors; every new vector is orthogonalised
// against the whole basis twice (so the projected matrix is formed from
// inner products, not assumed tridiagonal), Rayleigh-Ritz on that matrix gives
// the Ritz pairs of Q^2, and the basis restarts from the kk lowest Ritz
// vectors plus the last Lanczos vector (thick restart).  The converged Ritz
// vectors then get a Rayleigh-Ritz step with Q itself, which separates pairs
// +-lambda that Q^2 cannot.  Canonical layout, the caller's FP64 links.
// ---------------------------------------------------------------------------
struct LanczosOut {
  int restarts = 0;
  long long matvecs = 0;
  bool converged = false;
};

LanczosOut lanczos_q2(lq_ctx *c, const c128 *U, double m0, int n_eig, int n_want, int n_kv, double tol,
                      int max_restarts, const c128 *v0, double *lam, c128 *Vout, double *resid) {
  const long long V12 = 12LL * c->gcan.V;
  const Shifts z = shifts_of(nullptr, 0);
  c128 *B = c->lz_basis[0].get((size_t)(n_kv + 1) * V12);
  c128 *B2 = c->lz_basis[1].get((size_t)(n_kv + 1) * V12);
  c128 *tmp = c->lz_tmp.get((size_t)kMaxRhs * V12);
  LanczosOut out;
  auto at = [](std::vector<cd> &M, int n, int i, int j) -> cd & { return M[(size_t)i * n + j]; };
  // first basis vector
  copy<double>(c, B, v0, V12);
  {
    const double nv = norms<double>(c, B, V12, 1)[0];
    if (!(nv > 0)) fail(LQ_ERR_ARG, "lanczos_lowmodes: the start vector is zero");
    scale<double>(c, {cd(1.0 / nv)}, B, V12, B, V12, V12, 1, false);
  }
  std::vector<cd> T((size_t)n_kv * n_kv, cd(0));
  std::vector<double> theta;
  std::vector<cd> Z;
  std::vector<int> ord;
  double beta = 0;
  int k = 0;                 // vectors carried over from the last restart
  for (;;) {
    for (int j = k; j < n_kv; ++j) {
      c128 *vj = B + j * V12, *w = B + (j + 1) * V12;
      launch_wilson<double>(c->gcan, U, vj, tmp, nullptr, m0, z, 1, W_QSHIFT, c->st, clov_can(c));
      launch_wilson<double>(c->gcan, U, tmp, w, nullptr, m0, z, 1, W_QSHIFT, c->st, clov_can(c));
      ++out.matvecs;
      std::vector<cd> h1 = gram(c, j + 1, B, V12, 1, w, V12, V12);
      combine(c, j + 1, B, V12, 1, h1, -1.0, w, V12, V12, true);
      std::vector<cd> h2 = gram(c, j + 1, B, V12, 1, w, V12, V12);
      combine(c, j + 1, B, V12, 1, h2, -1.0, w, V12, V12, true);
      for (int i = 0; i <= j; ++i) {
        const cd t = h1[i] + h2[i];
        at(T, n_kv, i, j) = (i == j) ? cd(t.real(), 0.0) : t;
        at(T, n_kv, j, i) = (i == j) ? cd(t.real(), 0.0) : std::conj(t);
      }
      beta = norms<double>(c, w, V12, 1)[0];
      if (!(beta > 0)) fail(LQ_ERR_NUMERIC, "lanczos_lowmodes: the Krylov space became invariant");
      if (j + 1 < n_kv) {
        at(T, n_kv, j + 1, j) = at(T, n_kv, j, j + 1) = cd(beta);
        scale<double>(c, {cd(1.0 / beta)}, w, V12, w, V12, V12, 1, false);
      }
    }
    // Rayleigh-Ritz with Q^2 on the basis
    std::vector<cd> A = T;
    herm_eigh(n_kv, A, Z);
    theta.resize(n_kv);
    ord.resize(n_kv);
    for (int i = 0; i < n_kv; ++i) { theta[i] = A[(size_t)i * n_kv + i].real(); ord[i] = i; }
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return theta[a] < theta[b]; });
    // A B_i = sum_l B_l T_li (+ beta b_nkv for the last column): the residual of
    // Ritz pair i is beta |z_i[n_kv - 1]|; converged when it is below tol 2|lambda|
    int nconv = 0;
    for (int r = 0; r < n_want; ++r) {
      const int i = ord[r];
      const double res = beta * std::abs(Z[(size_t)(n_kv - 1) * n_kv + i]);
      const double lam_abs = std::sqrt(std::max(theta[i], 0.0));
      if (res <= tol * 2.0 * lam_abs) ++nconv;
      else break;
    }
    if (verbose())
      std::fprintf(stderr, "[lqmg] lanczos cycle %d: %d of %d converged, %lld Q^2 products\n", out.restarts, nconv,
                   n_want, out.matvecs);
    if (nconv >= n_want) { out.converged = true; break; }
    if (out.restarts >= max_restarts) break;
    // thick restart: the kk lowest Ritz vectors, then the last Lanczos vector
    const int kk = std::min(n_kv - 8, std::max(n_want + (n_kv - n_want) / 2, n_want + 1));
    for (int i0 = 0; i0 < kk; i0 += kMaxRhs) {
      const int nk = std::min(kMaxRhs, kk - i0);
      std::vector<cd> Y((size_t)n_kv * nk);
      for (int l = 0; l < n_kv; ++l)
        for (int q = 0; q < nk; ++q) Y[(size_t)l * nk + q] = Z[(size_t)l * n_kv + ord[i0 + q]];
      combine(c, n_kv, B, V12, nk, Y, 1.0, B2 + (long long)i0 * V12, V12, V12, false);
    }
    scale<double>(c, {cd(1.0 / beta)}, B + (long long)n_kv * V12, V12, B2 + (long long)kk * V12, V12, V12, 1,
                  false);
    std::fill(T.begin(), T.end(), cd(0));
    for (int i = 0; i < kk; ++i) {
      at(T, n_kv, i, i) = cd(theta[ord[i]]);
      const cd a = beta * Z[(size_t)(n_kv - 1) * n_kv + ord[i]];
      at(T, n_kv, kk, i) = a;
      at(T, n_kv, i, kk) = std::conj(a);
    }
    std::swap(B, B2);
    std::swap(c->lz_basis[0].p, c->lz_basis[1].p);
    std::swap(c->lz_basis[0].n, c->lz_basis[1].n);
    k = kk;
    ++out.restarts;
  }
  // Ritz vectors of the n_want lowest, then Rayleigh-Ritz with Q on them
  const int nw = n_want;
  for (int i0 = 0; i0 < nw; i0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, nw - i0);
    std::vector<cd> Y((size_t)n_kv * nk);
    for (int l = 0; l < n_kv; ++l)
      for (int q = 0; q < nk; ++q) Y[(size_t)l * nk + q] = Z[(size_t)l * n_kv + ord[i0 + q]];
    combine(c, n_kv, B, V12, nk, Y, 1.0, B2 + (long long)i0 * V12, V12, V12, false);
  }
  std::vector<cd> G((size_t)nw * nw);
  for (int j0 = 0; j0 < nw; j0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, nw - j0);
    launch_wilson<double>(c->gcan, U, B2 + (long long)j0 * V12, tmp, nullptr, m0, z, nk, W_QSHIFT, c->st,
                          clov_can(c));
    auto g = gram(c, nw, B2, V12, nk, tmp, V12, V12);
    for (int i = 0; i < nw; ++i)
      for (int q = 0; q < nk; ++q) G[(size_t)i * nw + j0 + q] = g[(size_t)i * nk + q];
  }
  for (int i = 0; i < nw; ++i)
    for (int j = i; j < nw; ++j) {
      const cd h = 0.5 * (G[(size_t)i * nw + j] + std::conj(G[(size_t)j * nw + i]));
      G[(size_t)i * nw + j] = h;
      G[(size_t)j * nw + i] = std::conj(h);
    }
  std::vector<cd> Zq;
  herm_eigh(nw, G, Zq);
  std::vector<double> mu(nw);
  std::vector<int> oq(nw);
  for (int i = 0; i < nw; ++i) { mu[i] = G[(size_t)i * nw + i].real(); oq[i] = i; }
  std::sort(oq.begin(), oq.end(), [&](int a, int b) { return std::fabs(mu[a]) < std::fabs(mu[b]); });
  for (int i0 = 0; i0 < n_eig; i0 += kMaxRhs) {
    const int nk = std::min(kMaxRhs, n_eig - i0);
    std::vector<cd> Y((size_t)nw * nk);
    for (int l = 0; l < nw; ++l)
      for (int q = 0; q < nk; ++q) Y[(size_t)l * nk + q] = Zq[(size_t)l * nw + oq[i0 + q]];
    c128 *X = Vout + (long long)i0 * V12;
    combine(c, nw, B2, V12, nk, Y, 1.0, X, V12, V12, false);
    // residuals ||Q x - lambda x||
    launch_wilson<double>(c->gcan, U, X, tmp, nullptr, m0, z, nk, W_QSHIFT, c->st, clov_can(c));
    std::vector<cd> a(nk);
    for (int q = 0; q < nk; ++q) {
      lam[i0 + q] = mu[oq[i0 + q]];
      a[q] = cd(-lam[i0 + q]);
    }
    scale<double>(c, a, X, V12, tmp, V12, V12, nk, true);
    auto r = norms<double>(c, tmp, V12, nk);
    for (int q = 0; q < nk; ++q) resid[i0 + q] = r[q];
  }
  return out;
}
}  // namespace

extern "C" {

int lma_low(lq_ctx *c, const lq_c128 *U, double m0, int n, const lq_c128 *V, const double *lam, const double *eps,
            double cutoff, double *loop_low, double *conn_low, int *n_kept) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !V || !lam || !eps || n < 1 || !(cutoff > 0)) fail(LQ_ERR_ARG, "lma_low: bad arguments");
    const int T = c->L[3];
    const long long Vol = c->gcan.V, V12 = 12LL * Vol;
    LmaLow L = lma_prepare(c, (const c128 *)U, m0, n, (const c128 *)V, lam, eps, cutoff);
    if (n_kept) *n_kept = L.n;
    std::vector<double> lr(2 * T, 0.0), cr(2 * T, 0.0);
    if (L.n > 0) {
      const int nn = L.n;
      // O[t][j][i] = sum over timeslice t of <v_j, v_i>
      std::vector<cd> O((size_t)T * nn * nn);
      c128 *dout = c->lma_out.get((size_t)T * nn * kMaxRhs);
      for (int k0 = 0; k0 < nn; k0 += kMaxRhs) {
        const int nk = std::min(kMaxRhs, nn - k0);
        launch_slice_products(nn, c->lma_V.p, nk, c->lma_V.p + k0 * V12, Vol, T, dout, c->st);
        std::vector<cd> h((size_t)T * nn * nk);
        LQ_HIP(hipMemcpyAsync(h.data(), dout, h.size() * sizeof(cd), hipMemcpyDeviceToHost, c->st));
        sync(c);
        for (int t = 0; t < T; ++t)
          for (int j = 0; j < nn; ++j)
            for (int k = 0; k < nk; ++k) O[((size_t)t * nn + j) * nn + k0 + k] = h[((size_t)t * nn + j) * nk + k];
      }
      // M(t) = A^{-1} O(t) (column by column through the LU factors)
      std::vector<cd> M((size_t)T * nn * nn), col(nn);
      for (int t = 0; t < T; ++t)
        for (int i = 0; i < nn; ++i) {
          for (int j = 0; j < nn; ++j) col[j] = O[((size_t)t * nn + j) * nn + i];
          lu_solve(nn, L.LU, L.piv, col.data());
          for (int j = 0; j < nn; ++j) M[((size_t)t * nn + j) * nn + i] = col[j];
        }
      // L_low(t) = tr M(t);  C_low(t) = (1/Vol) sum_t0 tr[M(t0) M(t0 + t)]
      for (int t = 0; t < T; ++t) {
        cd tr = 0;
        for (int i = 0; i < nn; ++i) tr += M[((size_t)t * nn + i) * nn + i];
        lr[2 * t] = tr.real();
        lr[2 * t + 1] = tr.imag();
      }
      for (int t = 0; t < T; ++t) {
        cd acc = 0;
        for (int t0 = 0; t0 < T; ++t0) {
          const cd *Ma = &M[(size_t)t0 * nn * nn], *Mb = &M[(size_t)((t0 + t) % T) * nn * nn];
          for (int i = 0; i < nn; ++i)
            for (int j = 0; j < nn; ++j) acc += Ma[(size_t)i * nn + j] * Mb[(size_t)j * nn + i];
        }
        acc /= (double)Vol;
        cr[2 * t] = acc.real();
        cr[2 * t + 1] = acc.imag();
      }
    }
    if (loop_low) std::memcpy(loop_low, lr.data(), lr.size() * sizeof(double));
    if (conn_low) std::memcpy(conn_low, cr.data(), cr.size() * sizeof(double));
    return LQ_OK;
  });
}

int lma_high(lq_ctx *c, const lq_c128 *U, double m0, int n, const lq_c128 *V, const double *lam, const double *eps,
             double cutoff, int n_noise, const lq_c128 *eta, double tol, double *loop_high) {
  return guard(c, [&] {
    need_mg(c);
    if (!U || !eta || !loop_high || n_noise < 1 || n < 0 || (n > 0 && (!V || !lam || !eps)) || !(tol > 0) ||
        !(cutoff > 0))
      fail(LQ_ERR_ARG, "lma_high: bad arguments");
    const int T = c->L[3];
    const long long Vol = c->gcan.V, V12 = 12LL * Vol;
    LmaLow L;
    if (n > 0) L = lma_prepare(c, (const c128 *)U, m0, n, (const c128 *)V, lam, eps, cutoff);
    c128 *R = c->lma_W.get((size_t)kMaxRhs * V12);     // R~ eta, then the solution
    c128 *X = c->lma_X.get((size_t)kMaxRhs * V12);
    c128 *b = c->tmpA.get((size_t)kMaxRhs * V12), *xb = c->tmpB.get((size_t)kMaxRhs * V12);
    c128 *dout = c->lma_out.get((size_t)T * kMaxRhs);
    std::vector<double> zs(kMaxRhs, 0.0);
    for (int k0 = 0; k0 < n_noise; k0 += kMaxRhs) {
      const int nk = std::min(kMaxRhs, n_noise - k0);
      const c128 *E = (const c128 *)eta + k0 * V12;
      copy<double>(c, R, E, (size_t)nk * V12);
      if (L.n > 0) {
        // R~ eta = eta - Q V A^{-1} V^dag eta
        auto cv = gram(c, L.n, c->lma_V.p, V12, nk, E, V12, V12);     // [n][nk]
        std::vector<cd> Y(cv.size()), col(L.n);
        for (int k = 0; k < nk; ++k) {
          for (int i = 0; i < L.n; ++i) col[i] = cv[(size_t)i * nk + k];
          lu_solve(L.n, L.LU, L.piv, col.data());
          for (int i = 0; i < L.n; ++i) Y[(size_t)i * nk + k] = col[i];
        }
        combine(c, L.n, c->lma_V.p, V12, nk, Y, 1.0, X, V12, V12, false);                 // X = V y
        launch_wilson<double>(c->gcan, (const c128 *)U, X, xb, R, m0, shifts_of(nullptr, 0), nk, W_RESID, c->st,
                              clov_can(c));
        copy<double>(c, R, xb, (size_t)nk * V12);                                        // R = eta - Q V y
      }
      // s = Q^{-1} R~ eta by the multigrid-preconditioned FGMRES (sigma = 0)
      launch_permute<double>(c->g, R, b, nk, true, c->st);
      int its[kMaxRhs];
      double rr[kMaxRhs];
      const bool ok = solve_shifted(c, nk, zs.data(), b, xb, tol, its, rr, c->p.fgmres_restarts);
      if (!ok) fail(LQ_ERR_NUMERIC, "lma_high: a deflated solve did not reach the tolerance");
      launch_permute<double>(c->g, xb, X, nk, false, c->st);
      // per timeslice: sum over t of eta_k^dag s_k
      for (int k = 0; k < nk; ++k) {
        launch_slice_products(1, E + k * V12, 1, X + k * V12, Vol, T, dout, c->st);
        std::vector<cd> h(T);
        LQ_HIP(hipMemcpyAsync(h.data(), dout, T * sizeof(cd), hipMemcpyDeviceToHost, c->st));
        sync(c);
        for (int t = 0; t < T; ++t) {
          loop_high[((size_t)(k0 + k) * T + t) * 2] = h[t].real();
          loop_high[((size_t)(k0 + k) * T + t) * 2 + 1] = h[t].imag();
        }
      }
    }
    return LQ_OK;
  });
}

int lanczos_lowmodes(lq_ctx *c, const lq_c128 *U, double m0, int n_eig, int n_guard, int n_kv, double tol,
                     int max_restarts, const lq_c128 *v0, double *lambda, lq_c128 *V, double *resid, int *info) {
  return guard(c, [&] {
    check_ctx(c);
    if (!U || !v0 || !lambda || !V || !resid || n_eig < 1 || n_guard < 0 || !(tol > 0) || max_restarts < 0)
      fail(LQ_ERR_ARG, "lanczos_lowmodes: bad arguments");
    const int n_want = n_eig + n_guard;
    if (n_kv > 191 || n_kv < n_want + 16)
      fail(LQ_ERR_ARG, "lanczos_lowmodes: need n_eig + n_guard + 16 <= n_kv <= 191");
    LanczosOut o = lanczos_q2(c, (const c128 *)U, m0, n_eig, n_want, n_kv, tol, max_restarts, (const c128 *)v0,
                              lambda, (c128 *)V, resid);
    if (info) {
      info[0] = o.restarts;
      info[1] = (int)std::min<long long>(o.matvecs, 0x7fffffff);
      info[2] = o.converged ? 1 : 0;
    }
    return LQ_OK;
  });
}

int lq_timeslice_products(lq_ctx *c, int nb, const lq_c128 *E, int nw, const lq_c128 *W, lq_c128 *out) {
  return guard(c, [&] {
    check_ctx(c);
    if (nb < 1 || nw < 1 || nw > kMaxRhs || !E || !W || !out) fail(LQ_ERR_ARG, "lq_timeslice_products: bad arguments");
    const int T = c->L[3];
    c128 *dout = c->lma_out.get((size_t)T * nb * nw);
    launch_slice_products(nb, (const c128 *)E, nw, (const c128 *)W, c->gcan.V, T, dout, c->st);
    LQ_HIP(hipMemcpyAsync(out, dout, (size_t)T * nb * nw * sizeof(c128), hipMemcpyDeviceToHost, c->st));
    sync(c);
    return LQ_OK;
  });
}

int mg_info(lq_ctx *c, int *nv, int *n_agg) {
  return guard(c, [&] {
    need_mg(c);
    if (nv) *nv = c->Nv;
    if (n_agg) *n_agg = c->cg.nA;
    return LQ_OK;
  });
}

int mg_info2(lq_ctx *c, int *nv2, int *n_agg2) {
  return guard(c, [&] {
    need_mg(c);
    if (c->n_levels != 3) fail(LQ_ERR_STATE, "the hierarchy has two levels");
    if (nv2) *nv2 = c->Nv2;
    if (n_agg2) *n_agg2 = c->cg2.nA;
    return LQ_OK;
  });
}

int mg_get_level2(lq_ctx *c, lq_c128 *P2, lq_c128 *Qc2) {
  return guard(c, [&] {
    need_mg(c);
    if (c->n_levels != 3) fail(LQ_ERR_STATE, "the hierarchy has two levels");
    if (P2) copy<double>(c, (c128 *)P2, c->P2_64.p, (size_t)c->Nv2 * c->cg.nA * c->cg.n2);
    if (Qc2) {
      const size_t n = (size_t)c->cg2.nA * 5 * c->cg2.n2 * c->cg2.n2;
      if (c->p.precision == LQ_PREC_FP64) copy<double>(c, (c128 *)Qc2, c->d64.Qc2.p, n);
      else launch_convert<double, float>(c->d32.Qc2.p, (c128 *)Qc2, (long long)n, c->st);
    }
    sync(c);
    return LQ_OK;
  });
}

int mg_get_interp(lq_ctx *c, lq_c128 *P) {
  return guard(c, [&] {
    need_mg(c);
    if (!P) fail(LQ_ERR_ARG, "NULL");
    launch_permute<double>(c->g, c->P64.p, (c128 *)P, c->Nv, false, c->st);
    sync(c);
    return LQ_OK;
  });
}

int mg_get_coarse(lq_ctx *c, lq_c128 *Qc) {
  return guard(c, [&] {
    need_mg(c);
    if (!Qc) fail(LQ_ERR_ARG, "NULL");
    const size_t n = (size_t)c->cg.nA * 5 * c->cg.n2 * c->cg.n2;
    if (c->p.precision == LQ_PREC_FP64) copy<double>(c, (c128 *)Qc, c->d64.Qc.p, n);
    else launch_convert<double, float>(c->d32.Qc.p, (c128 *)Qc, (long long)n, c->st);
    sync(c);
    return LQ_OK;
  });
}

// Component entry points run in the hierarchy's precision with FP64 interfaces.
int mg_restrict(lq_ctx *c, int n, const lq_c128 *f, lq_c128 *out) {
  return guard(c, [&] {
    need_mg(c);
    if (n < 1 || n > kMaxRhs || !f || !out) fail(LQ_ERR_ARG, "bad arguments");
    const long long V12 = 12LL * c->g.V, nc = (long long)c->cg.nA * c->cg.n2;
    c128 *fb = c->tmpA.get((size_t)kMaxRhs * V12);
    launch_permute<double>(c->g, (const c128 *)f, fb, n, true, c->st);
    if (c->p.precision == LQ_PREC_FP64) {
      launch_restrict<double>(c->g, c->d64.P.p, c->Nv, fb, V12, n, (c128 *)out, c->st);
    } else {
      c64 *f32 = c->f32a.get((size_t)n * V12);
      c64 *o32 = c->c32b.get((size_t)n * nc);
      launch_convert<float, double>(fb, f32, n * V12, c->st);
      launch_restrict<float>(c->g, c->d32.P.p, c->Nv, f32, V12, n, o32, c->st);
      launch_convert<double, float>(o32, (c128 *)out, n * nc, c->st);
    }
    sync(c);
    return LQ_OK;
  });
}

int mg_prolong(lq_ctx *c, int n, const lq_c128 *cin, lq_c128 *f) {
  return guard(c, [&] {
    need_mg(c);
    if (n < 1 || n > kMaxRhs || !cin || !f) fail(LQ_ERR_ARG, "bad arguments");
    const long long V12 = 12LL * c->g.V, nc = (long long)c->cg.nA * c->cg.n2;
    c128 *fb = c->tmpA.get((size_t)kMaxRhs * V12);
    if (c->p.precision == LQ_PREC_FP64) {
      launch_prolong<double>(c->g, c->d64.P.p, c->Nv, (const c128 *)cin, fb, V12, n, false, c->st);
    } else {
      c64 *c32 = c->c32b.get((size_t)n * nc);
      c64 *f32 = c->f32a.get((size_t)n * V12);
      launch_convert<float, double>((const c128 *)cin, c32, n * nc, c->st);
      launch_prolong<float>(c->g, c->d32.P.p, c->Nv, c32, f32, V12, n, false, c->st);
      launch_convert<double, float>(f32, fb, n * V12, c->st);
    }
    launch_permute<double>(c->g, fb, (c128 *)f, n, false, c->st);
    sync(c);
    return LQ_OK;
  });
}

int mg_coarse_apply(lq_ctx *c, int n, const double *sigma, const lq_c128 *x, lq_c128 *y) {
  return guard(c, [&] {
    need_mg(c);
    if (n < 1 || n > kMaxRhs || !sigma || !x || !y) fail(LQ_ERR_ARG, "bad arguments");
    const long long nc = (long long)c->cg.nA * c->cg.n2;
    Shifts S = shifts_of(sigma, n);
    if (c->p.precision == LQ_PREC_FP64) {
      launch_coarse_apply<double>(c->cg, c->d64.Qc.p, (const c128 *)x, (c128 *)y, S, n, false, c->st);
    } else {
      c64 *a = c->c32b.get((size_t)2 * n * nc);
      launch_convert<float, double>((const c128 *)x, a, n * nc, c->st);
      if (c->p.coarse_bf16)
        launch_coarse_apply_bf16(c->cg, c->QcB.p, a, a + n * nc, S, n, false, c->st);
      else
        launch_coarse_apply<float>(c->cg, c->d32.Qc.p, a, a + n * nc, S, n, false, c->st);
      launch_convert<double, float>(a + n * nc, (c128 *)y, n * nc, c->st);
    }
    sync(c);
    return LQ_OK;
  });
}

int mg_smooth(lq_ctx *c, int n, const double *sigma, const lq_c128 *r, lq_c128 *z, int steps) {
  return guard(c, [&] {
    need_mg(c);
    if (n < 1 || n > kMaxRhs || !sigma || !r || !z || steps < 0) fail(LQ_ERR_ARG, "bad arguments");
    const long long V12 = 12LL * c->g.V;
    c128 *rb = c->tmpA.get((size_t)kMaxRhs * V12), *zb = c->tmpB.get((size_t)kMaxRhs * V12);
    launch_permute<double>(c->g, (const c128 *)r, rb, n, true, c->st);
    smooth64(c, sigma, rb, zb, n, steps);
    launch_permute<double>(c->g, zb, (c128 *)z, n, false, c->st);
    sync(c);
    return LQ_OK;
  });
}

int mg_cycle(lq_ctx *c, int n, const double *sigma, const lq_c128 *r, lq_c128 *z) {
  return guard(c, [&] {
    need_mg(c);
    if (n < 1 || n > kMaxRhs || !sigma || !r || !z) fail(LQ_ERR_ARG, "bad arguments");
    const long long V12 = 12LL * c->g.V;
    c128 *rb = c->tmpA.get((size_t)kMaxRhs * V12), *zb = c->tmpB.get((size_t)kMaxRhs * V12);
    launch_permute<double>(c->g, (const c128 *)r, rb, n, true, c->st);
    precond64(c, sigma, rb, zb, n);
    launch_permute<double>(c->g, zb, (c128 *)z, n, false, c->st);
    sync(c);
    return LQ_OK;
  });
}

}  // extern "C"
