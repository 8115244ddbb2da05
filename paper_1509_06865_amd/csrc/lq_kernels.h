// Host-side launchers of the HIP kernels of liblqmg (one translation unit per
// kernel family).  All pointers are device pointers; all launches are
// asynchronous on the given stream.
#pragma once
#include "lq_common.h"
#include "lq_ktimer.h"

namespace lq {

struct Shifts { double s[kMaxRhs]; };

// ---- Wilson stencil (wilson.hip) -------------------------------------------
enum WilsonMode { W_QSHIFT = 0, W_RESID = 1 };
// mode W_QSHIFT: y_k = (Q - sigma_k) x_k ; W_RESID: y_k = b_k - (Q - sigma_k) x_k.
// C: the clover term [kCloverRows][V] in the layout of U (nullptr: none).
template <typename T>
void launch_wilson(const Geom &g, const cplx<T> *U, const cplx<T> *x, cplx<T> *y,
                   const cplx<T> *b, double m0, const Shifts &sig, int nrhs, int mode,
                   hipStream_t st, const cplx<T> *C = nullptr);
// Split hops of Q for the coarse operator.  Input: nf fields x (one column of
// P each) whose gamma5 half 'half[j]' is used (the other half read as zero).
// Output parts[j][5][12][V]: part 0 = gamma5[((4+m0) + C) x - 1/2 sum_mu (hops that
// stay inside a block)], part 1+mu = gamma5[-1/2 (forward mu hop leaving the block)].
template <typename T>
void launch_coarse_parts(const Geom &g, const cplx<T> *U, const cplx<T> *x, const int *half_dev,
                         int nf, long long xstride, cplx<T> *parts, double m0, hipStream_t st,
                         const cplx<T> *C = nullptr);
// Clover term of the FP64 links U (canonical or blocked, as g says) into
// C [kCloverRows][V] (clover.hip).
void launch_clover_build(const Geom &g, const c128 *U, double csw, c128 *C, hipStream_t st);

// ---- BLAS-1 (blas.hip) ------------------------------------------------------
// Batched vectors: nrhs vectors of length n, vector k at base + k*stride.
// Partial sums use a fixed reduction tree (deterministic).
// out[i][k] = <v_i,k , w_k> for i < nv (basis vector i of rhs k at
// vbase + i*vstride + k*rstride), w_k at w + k*wstride; vectors of n complex.
template <typename T>
void launch_dots(int nv, const cplx<T> *vbase, long long vstride, long long rstride,
                 const cplx<T> *w, long long wstride, long long n, int nrhs,
                 c128 *out /*device [nv][nrhs]*/, c128 *scratch, hipStream_t st,
                 const int *active = nullptr /*device [nrhs]: skip systems with 0*/);
// w_k += sign * sum_i h[i][k] v_i,k  (h device [nv][nrhs], FP64)
template <typename T>
void launch_multi_axpy(int nv, const cplx<T> *vbase, long long vstride, long long rstride,
                       const c128 *h, cplx<T> *w, long long wstride, long long n, int nrhs,
                       double sign, hipStream_t st, const int *active = nullptr);
// Device-side GMRES bookkeeping (blas.hip), one thread per system: see there.
void launch_arnoldi_start(int nrhs, int m, const c128 *nrm2, const double *bn, double tol, c128 *g, int *active,
                          int *kk, c128 *coef, hipStream_t st);
void launch_arnoldi_update(int j, int m, int nrhs, const c128 *h1, const c128 *h2, const c128 *nrm2, c128 *H,
                           double *cs, c128 *sn, c128 *g, const double *bn, double tol, int *active, int *kk,
                           c128 *coef, int *bad, hipStream_t st);
void launch_arnoldi_solve(int m, int nrhs, const c128 *H, const c128 *g, const int *kk, c128 *Y, hipStream_t st);
// ---- shared-basis products (gram.hip), FP64 -----------------------------------
// out[i][k] = <E_i, W_k> for i < nb (<= 192), k < nw (<= 16); E_i at E + i*estride,
// W_k at W + k*wstride, vectors of n complex.  FP64 MFMA, split over n.
// At most max_chunks element chunks (each leaves nb x 16 complex partial sums
// in scratch); the scratch must hold min(max_chunks, chunks for n) of them.
void launch_gram(int nb, const c128 *E, long long estride, int nw, const c128 *W, long long wstride, long long n,
                 c128 *out /*device [nb][nw]*/, c128 *scratch, hipStream_t st, long long max_chunks = 2048);
size_t gram_scratch_elems(long long n);
// complex partial sums one element chunk of the Gram kernel leaves for nb basis vectors
inline size_t gram_chunk_elems(int nb) { return (size_t)nb * 16; }
// out[t][i][k] = sum over timeslice t (canonical layout, t slowest) of <E_i, W_k>
// summed over the 12 components; nw <= 16, out device [T][nb][nw].
void launch_slice_products(int nb, const c128 *E, int nw, const c128 *W, long long V, int T, c128 *out,
                           hipStream_t st);
// U_k (+)= sum_i Y[i][k] E_i for k < nw; Y device [nb][nw].
void launch_combine(int nb, const c128 *E, long long estride, int nw, const c128 *Y, c128 *U, long long ustride,
                    long long n, bool accumulate, hipStream_t st);
// Scratch size (in c128 elements) that launch_dots needs.
size_t dots_scratch_elems(int nv, int nrhs);
// y_k = a_k * x_k (+ y_k if accumulate), a device [nrhs] c128
template <typename T>
void launch_scale(const c128 *a, const cplx<T> *x, long long xstride, cplx<T> *y, long long ystride,
                  long long n, int nrhs, bool accumulate, hipStream_t st);
// y = x with precision change
template <typename To, typename Ti>
void launch_convert(const cplx<Ti> *x, cplx<To> *y, long long n, hipStream_t st);
// canonical <-> blocked layout of [nf][12][V] fields
template <typename T>
void launch_permute(const Geom &blocked, const cplx<T> *x, cplx<T> *y, int nf, bool to_blocked,
                    hipStream_t st);
// links [4][9][V] canonical -> blocked with precision change
template <typename To>
void launch_pack_links(const Geom &blocked, const c128 *U, cplx<To> *out, hipStream_t st);

// ---- SAP (sap.hip) ----------------------------------------------------------
// One colour pass of multiplicative SAP on D_sigma = D - sigma gamma5 for
// rhs gamma5 r:  z_B += MR_B(gamma5 r - D_sigma z) on every block B of
// colour 'colour'.  Fields [nrhs][12][V] in the blocked layout (block = SAP block).
template <typename T>
void launch_sap_colour(const Geom &g, const cplx<T> *U, const cplx<T> *r, cplx<T> *z,
                       const int *blocks_of_colour, int nblocks, double m0, const Shifts &sig,
                       int nrhs, int n_mr, hipStream_t st, const cplx<T> *C = nullptr);

// ---- transfers (transfer.hip) -----------------------------------------------
// c[j][A][h*Nv + k] = sum_{x in A, s in h, col} conj(P_k[3s+col][x]) f_j[3s+col][x]
template <typename T>
void launch_restrict(const Geom &g, const cplx<T> *P, int Nv, const cplx<T> *f, long long fstride,
                     int nf, cplx<T> *c, hipStream_t st);
// f_j (+)= P c_j
template <typename T>
void launch_prolong(const Geom &g, const cplx<T> *P, int Nv, const cplx<T> *c, cplx<T> *f,
                    long long fstride, int nf, bool accumulate, hipStream_t st);
// P from Nv test vectors (FP64 fields [12][V], blocked; cols: device array
// of their addresses, so they need not be contiguous): per block and gamma5
// half, Cholesky-QR applied twice.  Writes P64 [Nv][12][V].  status (device
// int) set to 1 if a local Gram matrix is not positive definite.
void launch_build_P(const Geom &g, const c128 *const *cols, int Nv, c128 *P64, int *status, hipStream_t st);
// Q_c columns from restricted parts: parts_c[j][5][nA][2Nv] -> Qc[A][d][row][col_j]
template <typename T>
void launch_scatter_coarse(const cplx<T> *parts_c, int nf, const int *cols_host, int n2,
                           int nA, cplx<T> *Qc, hipStream_t st);

// ---- coarse level (coarse.hip) ------------------------------------------------
struct CoarseGeom {
  int nb[4];       // coarse lattice extents (blocks per direction)
  int nA;          // coarse sites
  int n2;          // 2 * Nv unknowns per coarse site
};
// A complex number stored as two bfloat16 (the upper 16 bits of an IEEE FP32):
// the optional storage of the FP32 coarse operator.
struct bf16c { unsigned short re, im; };
// out = bf16 of in (round to nearest even), n complex numbers
void launch_to_bf16(const cplx<float> *in, bf16c *out, long long n, hipStream_t st);
// as launch_coarse_apply<float> with Q_c stored in bfloat16 (FP32 arithmetic)
void launch_coarse_apply_bf16(const CoarseGeom &cg, const bf16c *Qc, const cplx<float> *x, cplx<float> *y,
                              const Shifts &sig, int nrhs, bool g5form, hipStream_t st, const double *dsig = nullptr);
int tune_coarse_apply_bf16(const CoarseGeom &cg, const bf16c *Qc, const cplx<float> *x, cplx<float> *y, int nrhs,
                           hipStream_t st);
// y_k = g5c^e (Q_c - sigma_k) x_k (e = 1 if gamma5c form); vectors [nrhs][nA][n2].
// sigma_k is read from the device array dsig[k] when dsig is given (a launch
// whose arguments do not change with the shifts, as graph replay needs), else
// from sig.  The kernel variant is the one tuned for the shape, if any.
template <typename T>
void launch_coarse_apply(const CoarseGeom &cg, const cplx<T> *Qc, const cplx<T> *x, cplx<T> *y,
                         const Shifts &sig, int nrhs, bool g5form, hipStream_t st, const double *dsig = nullptr);
// dst[k] = s.s[k] for k < n, in stream order
void launch_set_shifts(const Shifts &s, int n, double *dst, hipStream_t st);
// Time each coarse-apply variant on these operands (y is overwritten), keep the
// fastest for (precision, nA, n2, nrhs, device) and return it; a tuned shape
// returns its variant at once.  Synchronises the stream: never under capture.
template <typename T>
int tune_coarse_apply(const CoarseGeom &cg, const cplx<T> *Qc, const cplx<T> *x, cplx<T> *y, int nrhs,
                      hipStream_t st);
// the variant used for a shape: the forced one, else the tuned one, else -1
template <typename T>
int coarse_variant(const CoarseGeom &cg, int nrhs);
// force variant v (0..5) for every shape, or -1 to use the tuned choice; -1 return = bad v
int coarse_force_variant(int v);
// y_k = g5c x_k (elementwise)
template <typename T>
void launch_coarse_g5(const CoarseGeom &cg, const cplx<T> *x, cplx<T> *y, int nrhs, hipStream_t st);

// ---- third level (level2.hip) -----------------------------------------------------
// The lattice of aggregates (level 1, coarse sites canonical, x fastest) cut
// into blocks of extent b2 (level-2 aggregates).
struct Level2Geom {
  int nb1[4];      // level-1 lattice extents
  int b2[4];       // level-2 aggregate extents on it
  int nb2[4];      // level-2 lattice extents
  int nA1, nA2, bvol2;
  int Nv1, Nv2;    // test vectors per level (2 Nv unknowns per site)
};
// c2[j][A2][h Nv2 + k] = sum_{A1 in A2, c} conj(P2_k[A1][h Nv1 + c]) v_j[A1][h Nv1 + c]
template <typename T>
void launch_restrict2(const Level2Geom &g, const cplx<T> *P2, const cplx<T> *v, int nrhs, cplx<T> *c2,
                      hipStream_t st);
// v_j (+)= P2 c2_j
template <typename T>
void launch_prolong2(const Level2Geom &g, const cplx<T> *P2, const cplx<T> *c2, cplx<T> *v, int nrhs,
                     bool accumulate, hipStream_t st);
// P2 from level-1 test vectors W [Nv2][nA1][2 Nv1] (FP64): local CholQR twice per (A2, half);
// *status raised (block left as it was) where the vectors are dependent
void launch_build_P2(const Level2Geom &g, const c128 *W, c128 *P2, int *status, hipStream_t st);
// split couplings of Q_c applied to nc half-columns of P2: parts[q][5][nA1][2 Nv1]
template <typename T>
void launch_coarse_parts2(const Level2Geom &g, const cplx<T> *Qc, const cplx<T> *x, const int *half_dev, int nc,
                          long long xstride, cplx<T> *parts, hipStream_t st);

// ---- parallel-transport convolution (ptc.hip) ---------------------------------
// out[o] = sum_i sum_d W[o][i][d] T_d phi[i](. + d), canonical layout, FP64;
// phi [cin][12][V], W [cout][cin][81][4][4], out [cout][12][V]
// The same layer on the bfloat16 matrix cores (FP32 accumulation), 1 <= cin, cout <= 24;
// scratch: ptc_bf16_scratch_words(V, cin, cout) 32-bit words (bfloat16 weights and inputs).
size_t ptc_bf16_scratch_words(int V, int cin, int cout);
void launch_ptc_forward_bf16(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                             c128 *out, unsigned *scratch, hipStream_t st);
// The layer's gradients on the bfloat16 matrix cores (input gradient: the adjoint
// product; weight gradient: per-offset products summed over site chunks); gin or
// gW may be null; scratch: ptc_bf16_backward_scratch_words(V, cin, cout) words.
size_t ptc_bf16_backward_scratch_words(int V, int cin, int cout);
void launch_ptc_backward_bf16(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                              const c128 *gout, c128 *gin, c128 *gW, unsigned *scratch, hipStream_t st);
void launch_ptc_forward(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W, c128 *out,
                        hipStream_t st);
// gradients of a real loss through the layer (g = dL/dRe out + i dL/dIm out): gin [cin][12][V]
// and gW [cout][cin][81][4][4] in the same form; either may be null
void launch_ptc_backward(const Geom &g, const c128 *U, int cin, const c128 *phi, int cout, const c128 *W,
                         const c128 *gout, c128 *gin, c128 *gW, hipStream_t st);
// out[c] = phi[c] * relu(|phi[c](x)| + b[c]) / |phi[c](x)| (spin-colour norm per site); out may be phi
void launch_mod_relu(int V, int channels, const c128 *phi, const double *b, c128 *out, hipStream_t st);
// one Adam step (step number t >= 1) on n real values p with gradient g and moments m, v
void launch_adam(long long n, double *p, const double *g, double *m, double *v, double lr, double b1, double b2,
                 double eps, int t, hipStream_t st);
// training loss of outputs X [nout][12][V] for targets u [K][12][V] over aggregates of extents
// agg (canonical layout): part [2 * blocks] per-block values, *loss (device) their sum,
// gX (nullable) the gradient; nout, K <= 32; *status raised if the outputs are dependent
void launch_proj_loss(const int L[4], const int agg[4], int nout, const c128 *X, int K, const c128 *u, double *part,
                      double *loss, c128 *gX, int *status, hipStream_t st);
// gradients through it: gphi [channels][12][V], gb [channels]; scratch: channels * V doubles
void launch_mod_relu_backward(int V, int channels, const c128 *phi, const double *b, const c128 *gout, c128 *gphi,
                              double *gb, double *scratch, hipStream_t st);

}  // namespace lq
