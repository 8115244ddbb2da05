/*
 * lqmg.h -- C ABI of the MI355X eigensolver for the Hermitian Wilson-Dirac
 * operator Q = gamma5 D: Rayleigh quotient iteration whose shifted systems
 * (Q - sigma) are solved by FGMRES preconditioned with gamma5-preserving
 * aggregation multigrid.  Method: Bali et al., "(Approximate) Low-Mode
 * Averaging with a new Multigrid Eigensolver" (Lattice 2015), sec. 2, Alg. 1.
 *
 * Conventions (all calls):
 *   - lattice dims[4] = {X, Y, Z, T}; canonical site index
 *     n = x + X*(y + Y*(z + Z*t)) (x fastest); V = X*Y*Z*T.
 *   - gauge field U: device array [4][9][V] of complex (mu = x,y,z,t; entry
 *     3*a + b of U_mu(n), which maps colour b at n + mu_hat to colour a at n).
 *   - spinor field: device array [12][V] of complex, component 3*s + c
 *     (spin s, colour c); several fields stack as [n][12][V].
 *   - gamma basis: chiral, gamma5 = -g1 g2 g3 g4 = diag(1,1,-1,-1) (sec. 2);
 *     gamma_k = [[0, i sigma_k], [-i sigma_k, 0]], gamma_t = [[0,1],[1,0]].
 *   - D psi(n) = (4 + m0) psi(n) - 1/2 sum_mu [(1 - gamma_mu) U_mu(n) psi(n+mu)
 *                + (1 + gamma_mu) U_mu(n-mu)^dag psi(n-mu)], the t hop across
 *     the boundary multiplied by t_bc (-1 antiperiodic, +1 periodic).
 *   - device pointers are hipMalloc'd memory (e.g. torch tensors) on the
 *     device that was current at lq_create; the caller owns them.  The
 *     library never frees or keeps them past the call, except that mg_setup
 *     copies U (and the multigrid state derived from it) into context memory.
 *   - every call returns 0 on success, >0 when it completed with a warning
 *     (LQ_WARN_NOCONV: an iteration limit was reached; outputs hold the last
 *     iterate), <0 on error; lq_last_error() then describes it.
 *   - a context is bound to one stream and is not thread safe.  q_apply and
 *     q_apply_c64 are asynchronous on that stream; all other calls return
 *     after the device work they issued has completed.
 */
#ifndef LQMG_H
#define LQMG_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lq_ctx lq_ctx;
typedef struct { double re, im; } lq_c128;   /* layout of torch.complex128 */
typedef struct { float re, im; } lq_c64;     /* layout of torch.complex64  */

enum {
  LQ_OK = 0,
  LQ_WARN_NOCONV = 1,
  LQ_ERR_ARG = -1,     /* invalid argument: dims, sizes, aggregate shapes, NULL */
  LQ_ERR_STATE = -2,   /* call order: e.g. a solve before mg_setup */
  LQ_ERR_HIP = -3,     /* a HIP runtime call failed */
  LQ_ERR_OOM = -4,     /* device allocation failed */
  LQ_ERR_NUMERIC = -5  /* breakdown: non-finite values or a singular local basis */
};

enum { LQ_PREC_FP64 = 0, LQ_PREC_MIXED = 1 };   /* multigrid arithmetic */
enum { LQ_SMOOTH_SAP = 0, LQ_SMOOTH_GMRES = 1 };

/* Multigrid / solver parameters (sec. 2: mu, nu, smoother, coarse GMRES, the
 * FP64 FGMRES of sec. 2.2, the setup of sec. 2.1).  lq_params_default fills
 * the defaults; pass NULL to mg_setup to use them. */
typedef struct {
  int precision;        /* LQ_PREC_FP64: everything FP64; LQ_PREC_MIXED: the
                           multigrid preconditioner in FP32 under FP64 FGMRES */
  int smoother;         /* LQ_SMOOTH_SAP (SAP on D_sigma = gamma5 (Q - sigma)
                           with rhs gamma5 r) or LQ_SMOOTH_GMRES (GMRES on Q - sigma) */
  int pre;              /* mu: pre-smoothing steps (SAP sweeps or GMRES calls) */
  int post;             /* nu: post-smoothing steps */
  int sap_mr;           /* minimal-residual steps per SAP block solve */
  int gmres_smooth_m;   /* Krylov steps per GMRES smoother call */
  int coarse_m;         /* coarse GMRES restart length */
  int coarse_restarts;  /* coarse GMRES restarts after the first cycle */
  double coarse_tol;    /* coarse GMRES relative residual target */
  int fgmres_m;         /* outer FGMRES restart length */
  int fgmres_restarts;  /* outer FGMRES restarts after the first cycle */
  int n_init;           /* setup: smoother passes on the random start vectors */
  int n_setup;          /* setup: multigrid passes over the test vectors */
  int rqi_block;        /* RQI: shifted systems solved together (1..16) */
  int rqi_max_sweeps;   /* RQI: maximum passes over the unconverged vectors */
  double rqi_solve_tol; /* RQI: relative residual of each shifted solve */
  int rayleigh_ritz;    /* RQI: 1 = Rayleigh-Ritz over all vectors after each sweep */
  int rqi_guard;        /* RQI: vectors iterated beyond n_eig (guard band against
                           missed modes); the n_eig smallest |lambda| are returned */
  int rqi_solve_restarts; /* RQI: FGMRES restarts per shifted solve; RQI needs the
                           direction of (Q - sigma)^-1 v, not a small residual, and
                           near convergence the system is nearly singular */
  int rqi_deflate;      /* RQI: 1 = before each multigrid cycle, solve Q - sigma
                           exactly on the span of the current eigenvector
                           approximations (Galerkin correction, FP64) */
  int rqi_start_passes; /* RQI: passes of the setup's multigrid iteration (sec. 2.1)
                           over all start vectors before Alg. 1: v <- M_0 v with
                           the sigma = 0 preconditioner, re-orthonormalisation and
                           a Rayleigh-Ritz step; 0 = Alg. 1 from the start vectors
                           as given */
  int graphs;           /* 1 = the coarse GMRES replays the Arnoldi steps between
                           two convergence checks (8 steps) as one captured HIP
                           graph, cached per shape; same kernels and bitwise the
                           same results as 0 (direct launches, the default).
                           Off while LQ_KT_COARSE is timed */
  int coarse_bf16;      /* LQ_PREC_MIXED only: 1 = the FP32 multigrid reads Q_c
                           from a bfloat16 copy (8-bit mantissa, FP32 arithmetic
                           and accumulation): half the coarse operator's bytes,
                           a coarse operator accurate to ~2^-9 relative; the FP64
                           outer FGMRES keeps the solves exact.  0 = FP32 Q_c */
  /* three-level hierarchies only (n_levels = 3 in mg_setup): the level-1
     system is then solved by FGMRES (coarse_m, coarse_restarts, coarse_tol
     above) right-preconditioned by a level-1 two-grid cycle made of */
  int coarse2_m;        /* the level-2 GMRES (on the gamma5^c2 form): restart length */
  int coarse2_restarts; /* its restarts after the first cycle */
  double coarse2_tol;   /* its relative residual target; 0 = exactly coarse2_m steps
                           with no convergence test (no host synchronisation) */
  int smooth1_m;        /* GMRES steps per level-1 smoothing step (gamma5^c form; a
                           fixed number, no convergence test) */
  int post1;            /* level-1 post-smoothing steps after the level-2 correction */
  /* RQI solve effort for stragglers: a vector whose residual eps_i is below
     rqi_stall_eps and fell by less than half over its last sweep gets
     rqi_stall_restarts more FGMRES restarts in its next solve (its block is
     solved apart from the others); 0 = off.  Near convergence RQI with a
     loosely solved system converges linearly at the solve's residual
     reduction, so a vector that has stopped gaining needs a better solve */
  int rqi_stall_restarts;
  double rqi_stall_eps;
} lq_mg_params;

typedef struct {
  int iters[16];        /* FGMRES iterations per right-hand side */
  double relres[16];    /* final true relative residual per right-hand side */
  int coarse_iters;     /* total coarse GMRES iterations in the call */
} lq_solve_stats;

typedef struct {
  int sweeps;           /* passes of Alg. 1 over the unconverged vectors */
  int solves;           /* shifted systems solved */
  int fgmres_iters;     /* total FGMRES iterations */
  int p_rebuilds;       /* interpolation / coarse-operator rebuilds (not counted:
                           rebuilds in which the approximations were linearly
                           dependent on some aggregate, whose block of P then
                           kept its previous columns) */
  double t_solve, t_ortho, t_rebuild, t_rq;   /* seconds per phase */
} lq_rqi_stats;

int lq_params_default(lq_mg_params *p);

/* Create a context for a lattice.  dims: host int[4] (each >= 2); t_bc: -1
 * antiperiodic or +1 periodic in t; hip_stream: hipStream_t the context
 * issues all work on (NULL = default stream).  Errors: LQ_ERR_ARG. */
int lq_create(lq_ctx **out, const int dims[4], int t_bc, void *hip_stream);
int lq_destroy(lq_ctx *ctx);
const char *lq_last_error(const lq_ctx *ctx);

/* Clover term (sec. 2: the operator is the clover-improved Wilson operator):
 * from this call on, D = (4 + m0) + C(x) - 1/2 sum_mu (hops) in every operator
 * application of the context (q_apply, q_apply_c64, the multigrid, the
 * solves, RQI, the Krylov solver, LMA), with
 *   C(x) = csw (i/4) sum_{mu != nu} sigma_munu (x) F_munu(x),
 *   F_munu = (Q_munu - Q_munu^dag) / 8, Q_munu the four plaquettes of the
 *   mu-nu plane at x (all starting with +mu, then +nu), sigma_munu =
 *   (i/2)[gamma_mu, gamma_nu] in the chiral basis.
 * C is built from U (device [4][9][V] canonical FP64, the links the later
 * calls pass; gauge loops take no boundary sign) and held by the context.
 * csw = 0 returns to the plain Wilson operator (U may then be NULL).  The
 * hierarchy of an earlier mg_setup is dropped: call mg_setup afterwards.
 * Synchronous.  Errors: LQ_ERR_ARG, LQ_ERR_OOM. */
int lq_clover(lq_ctx *ctx, const lq_c128 *U, double csw);

/* y = Q x for n_rhs fields (sec. 2: Q = gamma5 D, with the clover term of
 * lq_clover if one is set).  U: device [4][9][V];
 * x, y: device [n_rhs][12][V], must not overlap.  Asynchronous.
 * Errors: LQ_ERR_ARG (NULL pointer, n_rhs < 1). */
int q_apply(lq_ctx *ctx, const lq_c128 *U, double m0, const lq_c128 *x,
            lq_c128 *y, int n_rhs);
/* Single-precision variant: same layouts with complex64 elements. */
int q_apply_c64(lq_ctx *ctx, const lq_c64 *U, double m0, const lq_c64 *x,
                lq_c64 *y, int n_rhs);

/* Adaptive multigrid setup (sec. 2.1) for Q(U, m0) with n_levels = 2 (the
 * paper's hierarchy) or 3 levels.  agg: host int[n_levels - 1][4]; agg[0] =
 * block extents of the fine aggregates (each divides the lattice extent; the
 * number of blocks per direction is 1 or even, so that red/black SAP is well
 * defined; at most 256 sites); agg[1] (three levels) = block extents of the
 * level-2 aggregates on the lattice of aggregates (each divides its extent).
 * n_tv: host int[n_levels - 1]; n_tv[0] = Nv test vectors (2*Nv coarse
 * unknowns per aggregate, 1 <= Nv <= min(32, 6*prod(agg[0]))); n_tv[1] = Nv2
 * of the third level (1 <= Nv2 <= min(32, Nv)): the level-2 test vectors are
 * the restrictions P^dag w of the first Nv2 vectors that build P (during RQI
 * the eigenvector approximations), orthonormalised per level-2 aggregate and
 * gamma5^c half.  tv0: device [n_tv[0]][12][V] random start vectors (the
 * method draws no random numbers itself).  p: NULL = defaults.  Copies U;
 * replaces any previous hierarchy.  After an error the context holds no
 * hierarchy (solve and RQI calls return LQ_ERR_STATE until a setup succeeds).
 * Start vectors that are linearly dependent on an aggregate (or level-2
 * aggregate) are an error; if the setup's multigrid passes make them so,
 * those aggregates keep their previous interpolation columns.
 * Errors: LQ_ERR_ARG, LQ_ERR_OOM, LQ_ERR_NUMERIC (locally dependent start vectors). */
int mg_setup(lq_ctx *ctx, const lq_c128 *U, double m0, int n_levels, const int n_tv[],
             const int agg[][4], const lq_c128 *tv0, const lq_mg_params *p);

/* Solve (Q - sigma[k]) x[k] = rhs[k] for k < n_rhs (1..16) to the relative
 * residual tol with FP64 flexible GMRES preconditioned by the multigrid cycle
 * (sec. 2.2).  sigma: host double[n_rhs]; rhs, x: device [n_rhs][12][V].
 * Uses the hierarchy as it stands (rqi_lowmodes rebuilds it from the
 * eigenvector approximations).  st: may be NULL.
 * Errors: LQ_ERR_STATE (no setup), LQ_ERR_ARG; LQ_WARN_NOCONV. */
int mg_solve_shifted(lq_ctx *ctx, int n_rhs, const double *sigma,
                     const lq_c128 *rhs, lq_c128 *x, double tol,
                     lq_solve_stats *st);

/* Lowest-|lambda| eigenpairs of Q by Alg. 1 (RQI + multigrid), to residual
 * ||Q v - lambda v|| <= tol with ||v|| = 1.  The iteration works on
 * n_work = n_eig + rqi_guard vectors.  Start vectors: the first min(Nv, n_work)
 * setup test vectors, then the n_v0 = n_work - min(Nv, n_work) device fields
 * V0 [n_v0][12][V]; if n_v0 == n_work, V0 replaces all start vectors (warm
 * start).  With rayleigh_ritz = 1 the vectors are replaced by the Ritz
 * vectors of their span after every sweep.  Stops when the n_eig vectors with
 * smallest |lambda| have converged.  Output: lambda, resid host
 * double[n_eig]; V device [n_eig][12][V]; sorted by (|lambda|, lambda).  The
 * hierarchy is left built from the eigenvector approximations.
 * Errors: LQ_ERR_STATE, LQ_ERR_ARG; LQ_WARN_NOCONV (sweep limit). */
int rqi_lowmodes(lq_ctx *ctx, int n_eig, double tol, double *lambda,
                 lq_c128 *V, double *resid, const lq_c128 *V0, int n_v0,
                 lq_rqi_stats *st);

/* Inner products out[i*nw + k] = <E_i, W_k> = sum_e conj(E_i[e]) W_k[e] of nb
 * device vectors E [nb][n] against nw device vectors W [nw][n] (complex128,
 * n elements each; 1 <= nb <= 192, 1 <= nw <= 16); out: host [nb][nw].  These
 * are the Gram-Schmidt / Rayleigh-Ritz products of Alg. 1 (sec. 2.1) and of
 * the projections A_ij = <v_i|Q|v_j> of sec. 3.2; FP64 matrix cores.
 * Errors: LQ_ERR_ARG. */
int lq_inner_products(lq_ctx *ctx, int nb, const lq_c128 *E, int nw, const lq_c128 *W,
                      long long n, lq_c128 *out);

/* ---- allocation-free variant ------------------------------------------------ */
/* Bytes of the fixed device array behind lq_inner_products_noalloc: one copy
 * per device, held until the process ends. */
#define LQ_NOALLOC_SCRATCH_BYTES (16 * 1024 * 1024)
/* For callers that cannot allocate device memory (work under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * products as lq_inner_products, with the same arguments, limits and errors,
 * computed without any device allocation.  Its partial sums and results live
 * in a fixed device array of LQ_NOALLOC_SCRATCH_BYTES per device; when n is
 * long the vectors are cut into fewer chunks than lq_inner_products uses
 * (at most (16 MiB - 64 KiB) / (256 * nb) of them), so the sums may differ by
 * rounding.  Every call on a device shares that device's array and leaves its
 * contents behind (no call depends on them): calls that overlap in time on
 * one device race, so issue them on one stream, one after another.  Returns
 * after the results are in out (host).  Errors: LQ_ERR_ARG, LQ_ERR_STATE (the
 * array's address could not be resolved for the device). */
int lq_inner_products_noalloc(lq_ctx *ctx, int nb, const lq_c128 *E, int nw, const lq_c128 *W,
                              long long n, lq_c128 *out);

/* ---- approximate low-mode averaging (sec. 3.2, 3.3) ------------------------- */
/* Low-mode parts from n approximate eigenpairs (lambda[i], V[i], eps[i]) of Q
 * (V: device [n][12][V] canonical, orthonormal; lambda, eps: host double[n]).
 * The pairs with eps_i <= cutoff |lambda_i| are kept (sec. 3.3); with A the
 * projected matrix <v_i|Q|v_j> of the kept ones, the low-mode inverse is
 * sum_ij (A^-1)_ij |v_i><v_j| (sec. 3.2).  Outputs per timeslice t (t slowest
 * in the site index; host double[2*T], re/im interleaved; either may be NULL):
 *   loop_low[t] = sum over the sites x of timeslice t of tr (Q~_low^-1)_{x,x};
 *   conn_low[t] = (1/V) sum over x, y with t_x - t_y = t (mod T) of
 *                 tr[(Q~_low^-1)_{x,y} (Q~_low^-1)_{y,x}];
 * n_kept (nullable): the number of pairs kept (at most 192).  Needs no
 * hierarchy.  Errors: LQ_ERR_ARG, LQ_ERR_NUMERIC (A singular). */
int lma_low(lq_ctx *ctx, const lq_c128 *U, double m0, int n, const lq_c128 *V, const double *lambda,
            const double *eps, double cutoff, double *loop_low, double *conn_low, int *n_kept);
/* High-mode part of the loop, one sample per noise field eta (device
 * [n_noise][12][V] canonical, e.g. Z2 + i Z2 noise): s = Q^-1 R~ eta with the
 * oblique projector R~ = 1 - Q V A^-1 V^dag of the kept pairs (sec. 3.2; all
 * pairs dropped or n = 0: R~ = 1), solved to the relative residual tol by
 * FGMRES with the context's multigrid (sigma = 0); loop_high[k][t] = sum over
 * timeslice t of eta_k^dag s_k (host double[n_noise][2*T], re/im).  The mean
 * over the noise of loop_high plus loop_low estimates the loop without bias
 * (Q~_low^-1 + Q^-1 R~ = Q^-1 for any approximations).  Needs mg_setup.
 * Errors: LQ_ERR_STATE, LQ_ERR_ARG, LQ_ERR_NUMERIC (a solve did not converge). */
int lma_high(lq_ctx *ctx, const lq_c128 *U, double m0, int n, const lq_c128 *V, const double *lambda,
             const double *eps, double cutoff, int n_noise, const lq_c128 *eta, double tol, double *loop_high);
/* out[t][i][k] = sum over timeslice t (and the 12 components) of conj(E_i) W_k
 * for canonical fields E [nb][12][V], W [nw][12][V] (device); out host
 * [T][nb][nw] c128; 1 <= nw <= 16.  The per-timeslice overlaps of sec. 3.2's
 * estimators.  Errors: LQ_ERR_ARG. */
int lq_timeslice_products(lq_ctx *ctx, int nb, const lq_c128 *E, int nw, const lq_c128 *W, lq_c128 *out);

/* ---- restarted Krylov eigensolver (the comparison of sec. 2.2) -------------- */
/* The n_eig eigenpairs of Q of smallest |lambda| by a restarted Lanczos
 * method on Q^2, the kind of solver the paper compares RQI with multigrid
 * against (sec. 2.2: a Krylov space of n_kv vectors, restarted from the
 * current approximations).  Each cycle extends the basis to n_kv vectors,
 * orthogonalising every new vector twice against the whole basis; the n_kv
 * x n_kv projected matrix gives Ritz pairs of Q^2, and the basis restarts from
 * the lowest Ritz vectors plus the last Lanczos vector.  A Ritz pair of Q^2
 * counts as converged when its residual is below tol * 2 sqrt(theta) (which
 * bounds the residual of Q by about tol); when the n_eig + n_guard lowest have
 * converged (or after max_restarts restarts), a Rayleigh-Ritz step with Q on
 * those n_eig + n_guard vectors separates pairs +-lambda, and the n_eig of
 * smallest |lambda| are returned.  U: device links [4][9][V] canonical as for
 * q_apply; v0: device start vector [12][V] (nonzero); V: device output
 * [n_eig][12][V] canonical; lambda, resid: host double[n_eig] (eigenvalues in
 * increasing |lambda|, residuals ||Q v - lambda v|| of the unit vectors);
 * info (nullable): host int[3] = restarts, Q^2 products, converged (0/1).
 * Needs no hierarchy; allocates 2 (n_kv + 1) + 16 fields.
 * n_eig + n_guard + 16 <= n_kv <= 191.  Errors: LQ_ERR_ARG, LQ_ERR_NUMERIC
 * (the Krylov space became invariant), LQ_ERR_OOM. */
int lanczos_lowmodes(lq_ctx *ctx, const lq_c128 *U, double m0, int n_eig, int n_guard, int n_kv, double tol,
                     int max_restarts, const lq_c128 *v0, double *lambda, lq_c128 *V, double *resid, int *info);

/* ---- learned setup: network layer (not part of the paper) ------------------- */
/* One parallel-transport convolution of the network that proposes multigrid
 * test vectors:  out[o](x) = sum_{i < c_in} sum_{d in {-1,0,1}^4}
 * W[o][i][d] T_d(x) phi[i](x + d), where T_d(x) is the product of the links
 * along the path from x to x + d through the directions x, y, z, t in that
 * order (U_mu(y) for a step +mu, U_mu(y - mu)^dag for a step -mu, the t
 * boundary sign for a step across it).  Offsets are numbered
 * k = sum_mu (d_mu + 1) 3^(3 - mu).  All pointers are device memory in the
 * canonical layout: U [4][9][V] as for q_apply, phi [c_in][12][V],
 * W [c_out][c_in][81][4][4] (spin matrices, row-major), out [c_out][12][V].
 * FP64, asynchronous on the context's stream.  1 <= c_in, c_out <= 64.
 * out must not overlap phi, U or W (every site reads its neighbours' phi).
 * Sizes cannot be checked here: the caller passes arrays of exactly these
 * shapes.  Errors: LQ_ERR_ARG. */
int lq_ptc_forward(lq_ctx *ctx, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out,
                   const lq_c128 *W, lq_c128 *out);
/* The same layer on the bfloat16 matrix cores: weights, inputs and path
 * products rounded to bfloat16 (8-bit mantissa), products accumulated in FP32
 * (v_mfma_f32_16x16x16bf16), output written as complex128.  The layer as a
 * product per offset d: M = 4 c_out rows (o, s), K = 4 c_in (i, t), N = 3 V
 * columns (x, colour).  Arguments and layouts as lq_ptc_forward;
 * 1 <= c_in, c_out <= 24; out must not overlap phi, U or W.  Allocates a
 * scratch of 81 (4 c_out) (4 c_in) + 12 c_in V words on first use.  The result
 * differs from lq_ptc_forward by the bfloat16 rounding (about 2^-9 relative
 * per entry).  Errors: LQ_ERR_ARG, LQ_ERR_OOM. */
int lq_ptc_forward_bf16(lq_ctx *ctx, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out,
                        const lq_c128 *W, lq_c128 *out);
/* Gradients through lq_ptc_forward for a real loss L: given g_out =
 * dL/dRe(out) + i dL/dIm(out) (device [c_out][12][V]), writes g_in (device
 * [c_in][12][V]) and g_W (device [c_out][c_in][81][4][4]) of the same form for
 * phi and W; either output may be NULL.  g_in is the adjoint convolution, g_W
 * sums over the sites in a fixed order.  FP64, asynchronous on the context's
 * stream.  g_in and g_W must not overlap each other or any input.
 * Errors: LQ_ERR_ARG. */
int lq_ptc_backward(lq_ctx *ctx, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out,
                    const lq_c128 *W, const lq_c128 *g_out, lq_c128 *g_in, lq_c128 *g_W);
/* The same gradients on the bfloat16 matrix cores: g_out, W and phi rounded
 * to bfloat16, the path products formed in FP32, products accumulated in
 * FP32.  g_in is the adjoint layer (M = 4 c_in rows (i, t), K = 4 c_out, the
 * conjugated weights and the back-transported g_out); g_W is, per offset, the
 * product of g_out (rows (o, s), K = 3 V) with the conjugated transported
 * inputs (columns (i, t)), summed by site chunks of about 2048 sites in FP32
 * and the chunk sums added in a fixed order in FP64.  Arguments, layouts and
 * aliasing rules as lq_ptc_backward; 1 <= c_in, c_out <= 24.  Allocates (on
 * first use, shared with lq_ptc_forward_bf16) a scratch of 12 (c_in + c_out) V
 * + 81 (4 c_in)(4 c_out) words + 2 n_chunks (the g_W size) floats.  The
 * results differ from lq_ptc_backward by the bfloat16 rounding.  Errors:
 * LQ_ERR_ARG, LQ_ERR_OOM. */
int lq_ptc_backward_bf16(lq_ctx *ctx, const lq_c128 *U, int c_in, const lq_c128 *phi, int c_out,
                         const lq_c128 *W, const lq_c128 *g_out, lq_c128 *g_in, lq_c128 *g_W);
/* The network's nonlinearity between layers (gauge invariant): for channel c
 * and site x, out[c](x) = phi[c](x) * max(|phi[c](x)| + b[c], 0) / |phi[c](x)|,
 * |.| the norm over the 12 spin-colour components (out = 0 where phi = 0).
 * phi, out: device [channels][12][V] (out may equal phi); b: device double
 * [channels].  Asynchronous on the context's stream.  1 <= channels <= 64.
 * Errors: LQ_ERR_ARG. */
int lq_mod_relu(lq_ctx *ctx, int channels, const lq_c128 *phi, const double *b, lq_c128 *out);
/* Gradients through lq_mod_relu for a real loss: from g_out (device
 * [channels][12][V], form as for lq_ptc_backward) writes g_phi (device, same
 * shape) and g_b (device double [channels], summed over the sites in a fixed
 * order).  Uses a context-owned scratch of channels * V doubles.  Errors:
 * LQ_ERR_ARG, LQ_ERR_OOM. */
int lq_mod_relu_backward(lq_ctx *ctx, int channels, const lq_c128 *phi, const double *b,
                         const lq_c128 *g_out, lq_c128 *g_phi, double *g_b);

/* Training loss of the network's outputs: for each aggregate (extents agg,
 * host int[4], dividing the lattice) and gamma5 half, the part of the targets
 * u that the span of the outputs X does not represent,
 *   loss = (1/K) sum_k sum_{A,h} || (1 - Pi_{A,h}) u_k ||^2,
 * and (if g_X is not NULL) its gradient with respect to X in the form of
 * lq_ptc_backward.  X: device [n_out][12][V], u: device [K][12][V] (canonical
 * layout), 1 <= n_out, K <= 32, n_out <= 6 * prod(agg).  loss: host double.
 * Synchronous.  Errors: LQ_ERR_ARG; LQ_ERR_NUMERIC if the outputs are
 * linearly dependent on an aggregate half. */
int lq_proj_loss(lq_ctx *ctx, const int agg[4], int n_out, const lq_c128 *X, int K, const lq_c128 *u,
                 double *loss, lq_c128 *g_X);

/* One Adam step for the network's training: on n real values (a complex
 * parameter counts as its real and imaginary parts) with gradient g and
 * moment estimates m, v (updated in place; zero before the first step),
 *   m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
 *   p -= lr / (1 - b1^t) * m / (sqrt(v / (1 - b2^t)) + eps),
 * t >= 1 the step number.  All arrays device double.  Asynchronous on the
 * context's stream.  Errors: LQ_ERR_ARG. */
int lq_adam_step(lq_ctx *ctx, long long n, double *p, const double *g, double *m, double *v, double lr,
                 double beta1, double beta2, double eps, int t);

/* ---- dense helper ----------------------------------------------------------- */
/* Eigen-decomposition of the Hermitian part of the n x n matrix A (host,
 * row-major): w[j] ascending, V (host, row-major) holds the orthonormal
 * eigenvectors as columns, A V = V diag(w).  The Rayleigh-Ritz step of the
 * eigensolver (the projected problem V^dag Q V of Alg. 1's iterates) uses this
 * routine (Householder tridiagonalisation, implicit QL).  No context, no
 * device.  Errors: LQ_ERR_ARG. */
int lq_herm_eigh(int n, const lq_c128 *A, double *w, lq_c128 *V);

/* ---- coarse-apply kernel choice --------------------------------------------- */
/* The coarse operator apply (sec. 2's Q_c acting on coarse vectors) has eight
 * kernels: 0 one wavefront per (coarse site, rhs); 1, 2, 3 one workgroup per
 * coarse site with each 2Nv x 2Nv block staged in LDS and applied to 4, 8 or
 * 16 right-hand sides per pass; 4, 5 as 1, 2 with one workgroup per (coarse
 * site, chunk of 4 or 8 right-hand sides); 6 the matrix-core kernel (FP32
 * arithmetic on FP32 or bfloat16 storage, one workgroup per (coarse site,
 * 16 right-hand sides), 2Nv a multiple of 8 up to 64; where it does not apply
 * kernel 2 runs instead); 7 the matrix-core kernel on bfloat16 operands with
 * FP32 accumulation (bfloat16 storage only, i.e. coarse_bf16 = 1; the fields
 * are rounded to bfloat16 inside the kernel; same block sizes as 6; where it
 * does not apply kernel 6 runs instead).  By default each coarse solve times
 * the applicable kernels on its first call for a shape (precision, storage,
 * coarse sites, 2Nv, rhs count, device) and keeps the fastest for the process.
 * lq_coarse_variant(v) with v in 0..7 forces kernel v for every shape (tests
 * compare them); v = -1 returns to the tuned choice.  Process-wide, not
 * thread-safe.  Errors: LQ_ERR_ARG for v outside -1..7. */
int lq_coarse_variant(int v);

/* ---- kernel timing (measurement of the hot kernels against the roofline) -- */
/* Kernel classes: 0 Wilson stencil (q_apply and the solves), 1 SAP colour
 * passes, 2 restriction, 3 prolongation, 4 coarse operator apply, 5 Gram
 * products, 6 basis combinations; -1 switches timing off. */
enum { LQ_KT_OFF = -1, LQ_KT_WILSON = 0, LQ_KT_SAP = 1, LQ_KT_RESTRICT = 2, LQ_KT_PROLONG = 3,
       LQ_KT_COARSE = 4, LQ_KT_GRAM = 5, LQ_KT_COMBINE = 6 };
/* Start timing one kernel class (process-wide, all contexts; clears earlier
 * totals).  While on, every launch of the class records a pair of HIP events
 * on the stream it is launched on and adds its algorithmic bytes (the data it
 * must move at least: every operand read once, every result written once).
 * Not thread-safe.  Errors: LQ_ERR_ARG for an unknown class. */
int lq_kernel_timer_start(int kind);
/* Launches timed since the last start, the sum of their device durations in
 * milliseconds and of their algorithmic bytes; waits for the recorded events.
 * Any argument may be NULL.  Errors: LQ_ERR_HIP. */
int lq_kernel_timer_read(long long *launches, double *ms_total, double *bytes_total);

/* ---- inspection of the hierarchy (parity tests; sec. 2 objects) ---------- */
/* Number of test vectors Nv and aggregates nA of the current hierarchy. */
int mg_info(lq_ctx *ctx, int *nv, int *n_agg);
/* P as Nv canonical fields: device [Nv][12][V] c128; restricted to aggregate
 * A and gamma5 half h the fields give the orthonormal columns (A, h, k). */
int mg_get_interp(lq_ctx *ctx, lq_c128 *P);
/* Q_c = P^dag Q P: device [nA][5][2Nv][2Nv] c128, block 0 = aggregate with
 * itself, block 1 + mu = aggregate A with A + mu_hat (row index h*Nv + k of A,
 * column index of the neighbour); the A - mu blocks are the conjugate
 * transposes of the A - mu forward blocks (Q_c is Hermitian). */
int mg_get_coarse(lq_ctx *ctx, lq_c128 *Qc);
/* Third level: Nv2 and the number nA2 of level-2 aggregates (LQ_ERR_STATE
 * for a two-level hierarchy). */
int mg_info2(lq_ctx *ctx, int *nv2, int *n_agg2);
/* The third level's P2 as Nv2 level-1 vectors, device [Nv2][nA][2Nv] c128
 * (restricted to level-2 aggregate A2 and gamma5^c half h they give the
 * orthonormal columns (A2, h, k)), and Q_c2 = P2^dag Q_c P2, device
 * [nA2][5][2Nv2][2Nv2] c128 in the layout of mg_get_coarse (level-2 lattice:
 * the lattice of aggregates cut into blocks agg[1], x fastest).  Either may
 * be NULL.  Errors: LQ_ERR_STATE (two levels). */
int mg_get_level2(lq_ctx *ctx, lq_c128 *P2, lq_c128 *Qc2);
/* Restriction c = P^dag f: f device [n][12][V], c device [n][nA][2Nv]. */
int mg_restrict(lq_ctx *ctx, int n, const lq_c128 *f, lq_c128 *c);
/* Prolongation f = P c (shapes as above). */
int mg_prolong(lq_ctx *ctx, int n, const lq_c128 *c, lq_c128 *f);
/* y = (Q_c - sigma[k]) x[k] on coarse vectors [n][nA][2Nv]; sigma host.  In
 * mixed precision this is the stored FP32 (or, with coarse_bf16, bfloat16)
 * operator applied in FP32. */
int mg_coarse_apply(lq_ctx *ctx, int n, const double *sigma, const lq_c128 *x,
                    lq_c128 *y);
/* z = smoother applied to r for shifts sigma (steps as in the parameters'
 * 'post'): SAP on D_sigma with rhs gamma5 r from z = 0.  Shapes [n][12][V]. */
int mg_smooth(lq_ctx *ctx, int n, const double *sigma, const lq_c128 *r,
              lq_c128 *z, int steps);
/* z = B_sigma r, one multigrid cycle (eq. E_2g).  Shapes [n][12][V]. */
int mg_cycle(lq_ctx *ctx, int n, const double *sigma, const lq_c128 *r,
             lq_c128 *z);

#ifdef __cplusplus
}
#endif
#endif /* LQMG_H */
