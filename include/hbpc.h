/*
 * libhbpc -- HBPC(q, k_max) two-derivative deferred-correction time stepping
 * of the DGSEM on uniform periodic Cartesian meshes, for one AMD MI355X GPU.
 *
 * Method: Zeifang & Schuetz, "Two-derivative deferred correction time
 * discretization for the discontinuous Galerkin method" (arXiv 2109.04804).
 *
 * Conventions used by every entry point
 * -------------------------------------
 *  - State layout: w[e][v][node], contiguous, FP64 unless the name ends in
 *    _f32.  node = i + (N+1)(j + (N+1)k); elements are lexicographic with x
 *    fastest; v runs over the nvar conserved variables (advection and Burgers
 *    1, Euler d+2: rho, rho v_1..rho v_d, E).
 *  - ndof = n_elem (N+1)^d nvar (hbpc_ndof).  Extended vectors X = (w, sigma)
 *    hold the w block followed by the sigma block (2 ndof values).
 *  - All data pointers are DEVICE pointers owned by the caller, unless stated
 *    otherwise.  Input and output buffers must not overlap.
 *  - residual/JVP/preconditioner calls are asynchronous on the context's
 *    stream (hbpc_params.stream, or hbpc_set_stream); hbpc_step synchronises.
 *  - Return value 0 on success, a negative HBPC_ERR_* code otherwise; no
 *    exception crosses the ABI.  hbpc_last_error gives a message.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef HBPC_H
#define HBPC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hbpc_ctx hbpc_ctx;

/* error codes */
#define HBPC_OK 0
#define HBPC_ERR_ARG (-1)          /* invalid argument or unsupported combination */
#define HBPC_ERR_OOM (-2)          /* device allocation failed */
#define HBPC_ERR_HIP (-3)          /* HIP runtime error */
#define HBPC_ERR_NONFINITE (-4)    /* NaN/Inf in a residual norm */
#define HBPC_ERR_NEWTON (-5)       /* Newton did not converge within newton_maxit */
#define HBPC_ERR_GMRES (-6)        /* GMRES did not reach gmres_rtol within gmres_maxit */
#define HBPC_ERR_UNSUPPORTED (-7)  /* (dim, N, equation) not compiled in */

/* equations (Sec. 4.1.1 advection, Eq. Euler; viscous Burgers with BR1) */
#define HBPC_EQ_ADVECTION 1
#define HBPC_EQ_BURGERS_BR1 2
#define HBPC_EQ_EULER 3
#define HBPC_EQ_NAVIER_STOKES 4    /* Sec. 5.1: eps-scaled Euler flux minus the viscous flux, BR2 lifting
                                      (d = 2 with N <= 7, d = 3 with N <= 4) */

/* interpolation/quadrature nodes (Sec. 3.1.1 uses Gauss-Legendre) */
#define HBPC_NODES_GAUSS 0
#define HBPC_NODES_LOBATTO 1

/* numerical flux (Eq. Riemann): f* = (F(wL)+F(wR)).n/2 + lambda (wL - wR)/2 */
#define HBPC_FLUX_CENTRAL 0        /* lambda = 0 */
#define HBPC_FLUX_UPWIND 1         /* lambda = |a.n| (advection) */
#define HBPC_FLUX_LF 2             /* lambda = params.lambda, a global constant */
#define HBPC_FLUX_RUSANOV 3        /* lambda = max(|vL.n| + cL/eps, |vR.n| + cR/eps) (Euler) */
#define HBPC_FLUX_LF_LITERAL 4     /* Euler: Eq. Riemann as printed, lambda_v (wL - wR) without the 1/2,
                                      lambda = diag(1/eps, 1, .., 1, 1/eps) (Sec. 4.1.2 set-up) */

/* precision of the Krylov solve */
#define HBPC_FP64 0                /* everything FP64 */
#define HBPC_MIXED 1               /* FP64 Newton residual/updates, FP32 Krylov, JVP and BJ_ext */

/* preconditioner */
#define HBPC_PC_NONE 0
#define HBPC_PC_BJEXT 1            /* extended block-Jacobi, Sec. 3.2.3 */
#define HBPC_PC_LEARNED 2          /* per-element network on the Schur system (an addition to
                                      the paper, see hbpc_mlp_*), BJ_ext as fallback */
#define HBPC_PC_LEARNED_GUESS 4    /* the network's correction of the Newton residual as the
                                      initial guess of each Newton step's FGMRES (kept only if it
                                      lowers the residual norm), BJ_ext for every direction */
#define HBPC_PC_LEARNED_FIRST 3    /* flexible GMRES with the network for the first direction of
                                      each Newton step (z_0 = N(v_0), v_0 the normalised Newton
                                      residual: the network's training input) and BJ_ext for
                                      every later one; a non-finite network output drops the
                                      network for the rest of the stage solve (counted in
                                      pc_fallbacks) */
#define HBPC_PC_BJEXT_H 5          /* BJ^H_ext, Sec. 3.2.3: BJ_ext with the element-local
                                      Hessian block dR2/dw kept in P, built at the (w, sigma) of
                                      the Newton iterate at which pc_rebuild builds (FP64 blocks K
                                      and H; S^-1 stored as for BJ_ext) */

/* arithmetic of the learned preconditioner's network */
#define HBPC_MLP_BF16 0            /* BF16 operands on the matrix cores, FP32 accumulation */
#define HBPC_MLP_FP32 1            /* FP32 throughout (check path) */

/* preconditioner rebuild frequency */
#define HBPC_PC_PER_SOLVE 0        /* once per stage solve, at the Newton initial guess */
#define HBPC_PC_PER_NEWTON_IT 1    /* at every Newton iterate */
#define HBPC_PC_PER_STAGE 2        /* predictor: once per stage solve; corrector: once per stage in
                                      the first sweep, kept and reused by the later sweeps (same
                                      coefficients alpha1 dt = dt, alpha2 dt^2/2 = dt^2/2; the
                                      state has moved by one sweep's correction).  Keeps s - 1
                                      sets of S^-1 blocks. */
#define HBPC_PC_ACROSS_STEPS 3     /* the blocks of every predictor substep and corrector stage
                                      kept across time steps (Sec. 4.1.2 suggests reusing the
                                      preconditioner over several Newton steps or time steps):
                                      built on first use, rebuilt after pc_reuse_steps steps or
                                      when the solve's coefficients (dt) change.  Keeps 2 (s - 1)
                                      sets of S^-1 blocks, so q <= 6. */
#define HBPC_PC_PAIRED 4           /* corrector stages solved in pairs (their equations are
                                      independent, Alg. 1): the Newton and FGMRES iterations of two
                                      stages advance in lock step, the S^-1 blocks built at the first
                                      stage's state in the first sweep serve both stages and every
                                      later sweep, and one pass over the blocks applies them to the
                                      four right-hand sides of an iteration; the predictor as
                                      HBPC_PC_PER_SOLVE.  BJ_ext or HBPC_PC_LEARNED (each stage
                                      solve starts on the network and falls back to the shared
                                      blocks), with the linearised JVP only. */

/* Jacobian-vector product */
#define HBPC_JVP_LINEARISED 0      /* exact directional derivatives (hyper-dual flux) */
#define HBPC_JVP_FD 1              /* finite differences, Eq. MatrixFree_nonlinear (FP64 only) */

typedef struct {
    int dim;              /* 1, 2 or 3 */
    int nelem[3];         /* elements per direction (entries beyond dim ignored) */
    double length[3];     /* domain length per direction */
    double origin[3];     /* lower corner */
} hbpc_mesh;

typedef struct {
    int nodes;            /* HBPC_NODES_* */
    int flux;             /* HBPC_FLUX_* */
    double lambda;        /* constant lambda for HBPC_FLUX_LF */
    double adv[3];        /* advection velocity (HBPC_EQ_ADVECTION) */
    double nu;            /* viscosity (HBPC_EQ_BURGERS_BR1) */
    double gamma;         /* ratio of specific heats (Euler) */
    double eps_ref;       /* reference Mach number eps (Euler, Eq. Euler) */
    double mu;            /* dynamic viscosity (HBPC_EQ_NAVIER_STOKES, Eq. NavierStokes; default 0) */
    double prandtl;       /* Prandtl number (Navier-Stokes; default 0.72): heat conductivity
                             c_p mu / Pr with c_p = R gamma / (gamma - 1), R = 1 / (gamma eps^2) */
    double eta_br2;       /* BR2 stabilisation of the face gradients (Navier-Stokes; default 2):
                             face gradient = broken gradient + eta_br2 x the face's local lifting */
    int q;                /* quadrature order of the tableau: 4, 6 or 8 (appendix) */
    int kmax;             /* corrector sweeps k_max */
    double newton_rtol;   /* eps_N: stop when ||G(X^r)|| <= eps_N ||G(X^0)|| */
    double newton_atol_dw;/* ... or when ||dw^r||_2 / sqrt(ndof) <= this (default 1.95e-15):
                             the paper's absolute Newton tolerance ||dw||_2 <= 1e-12 (Sec. 5.2,
                             for 262,144 coefficients) taken per coefficient, so that it stays
                             above the round-off floor at every problem size; ... or, from the
                             second iteration on, when ||G(X^r)|| > 0.5 ||G(X^(r-1))|| and
                             ||dw^r||_2 <= 1e-12 ||w^0||_2 (the residual has reached the rounding
                             floor of its FP64 evaluation; counted in newton_floor_stops) */
    int newton_maxit;     /* default 30 */
    double gmres_rtol;    /* eps_G: stop when ||r_j|| <= eps_G ||r_0|| */
    int gmres_restart;    /* m of GMRES(m), 1..HBPC_MAX_RESTART (the paper restarts after 700
                             iterations, Sec. 4.1.2); the library keeps m + 1 basis vectors and m
                             preconditioned ones of 2 ndof values each (FP32 in HBPC_MIXED) */
    int gmres_maxit;      /* per Newton step (default 7000) */
    int precision;        /* HBPC_FP64 | HBPC_MIXED */
    int precond;          /* HBPC_PC_* */
    int pc_rebuild;       /* HBPC_PC_PER_SOLVE | HBPC_PC_PER_NEWTON_IT | HBPC_PC_PER_STAGE |
                             HBPC_PC_ACROSS_STEPS | HBPC_PC_PAIRED */
    int jvp_mode;         /* HBPC_JVP_* */
    int hessian;          /* 1: include dR2/dw in the JVP (exact Newton), 0: drop it */
    int mlp_precision;    /* HBPC_MLP_BF16 | HBPC_MLP_FP32: network arithmetic of HBPC_PC_LEARNED */
    double pc_fallback;   /* HBPC_PC_LEARNED: if a restart cycle of FGMRES ends with
                             ||r|| > pc_fallback ||r at the cycle's start||, or the network output
                             is not finite, the cycle's correction is dropped and BJ_ext takes over
                             for the rest of the stage solve (default 0.5; <= 0 never falls back) */
    int pc_half;          /* HBPC_MIXED: 1 stores the BJ_ext blocks S^-1 in FP16 (formed and inverted
                             in FP32, rounded once; the apply sums in FP32): half the bytes of the
                             apply.  An entry beyond the FP16 range makes the build fail with
                             HBPC_ERR_NONFINITE.  Default 0. */
    int pc_reuse_steps;   /* HBPC_PC_ACROSS_STEPS: time steps per set of blocks (>= 1, default 4) */
    int pc_probe_its;     /* HBPC_PC_LEARNED: length of the network's first restart cycle in each
                             stage solve (0, the default: gmres_restart).  A shorter probe is
                             judged by the same mean reduction per iteration: fallback when
                             ||r|| > pc_fallback^(pc_probe_its / gmres_restart) ||r at its start||.
                             Later cycles have the full length. */
    void* stream;         /* hipStream_t; NULL = the null stream */
} hbpc_params;

#define HBPC_MAX_SOLVES 64
/* largest FGMRES restart length (hbpc_params.gmres_restart) */
#define HBPC_MAX_RESTART 1024
typedef struct {
    int n_solves;                               /* stage solves in the last step */
    int newton_its;                             /* total Newton iterations */
    int gmres_its;                              /* total Krylov iterations */
    int pc_builds;                              /* BJ_ext builds */
    int newton_per_solve[HBPC_MAX_SOLVES];
    int gmres_per_solve[HBPC_MAX_SOLVES];
    double t_step_ms;                           /* wall time of the step (host clock) */
    double t_pc_build_ms, t_gmres_ms, t_residual_ms;  /* phase times (host clock, synchronised) */
    int pc_fallbacks;                           /* stage solves where BJ_ext replaced the learned PC */
    int mlp_samples;                            /* training samples collected during the step */
    int newton_floor_stops;                     /* Newton solves ended by the rounding-floor test */
} hbpc_stats;

/* Fill *p with the defaults: Gauss nodes, Rusanov flux, gamma 1.4, eps 1,
 * HBPC(6,4), eps_N 1e-8, atol_dw 1.95e-15 (RMS), 30 Newton its, eps_G 1e-3,
 * GMRES(30), 7000 its, FP64, BJ_ext per solve, linearised JVP with Hessian,
 * BF16 network, learned-preconditioner fallback ratio 0.5. */
void hbpc_default_params(hbpc_params* p);

/* Create a context: mesh (host struct), degree N (2..7 in 1-D and 2-D, 2..5 in 3-D; other
 * degrees return HBPC_ERR_UNSUPPORTED), equation HBPC_EQ_*.
 * Computes the 1-D operators (Sec. 3.1.1) on the host and allocates all
 * device work space (stage vectors, Krylov bases, BJ_ext blocks).  *out is
 * owned by the caller and released by hbpc_destroy.
 * Errors: HBPC_ERR_ARG, HBPC_ERR_UNSUPPORTED, HBPC_ERR_OOM, HBPC_ERR_HIP. */
int hbpc_create(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* params, hbpc_ctx** out);
int hbpc_destroy(hbpc_ctx* ctx);
int hbpc_set_stream(hbpc_ctx* ctx, void* stream);
size_t hbpc_ndof(const hbpc_ctx* ctx);
/* Element block size ne = nvar (N+1)^d. */
int hbpc_block_size(const hbpc_ctx* ctx);
/* 1-D nodes and weights into HOST arrays of N+1 doubles. */
int hbpc_nodes(const hbpc_ctx* ctx, double* xi_host, double* w_host);

/* R1_h(w) -> r1 (Eq. DGSEM_wt). */
int hbpc_residual1(hbpc_ctx* ctx, const double* w, double* r1);
/* For callers that cannot allocate device memory (code under stream capture, tight serving
 * loops, hosts that forbid hipMalloc): R1_h(w) -> r1 as hbpc_residual1 computes it, with no
 * context and no allocation of any kind.  mesh, params: host structs as for hbpc_create
 * (only the mesh, nodes, flux and equation parameters and params->stream are used); w, r1:
 * caller-owned device arrays of ndof doubles in the layout of hbpc_residual1, enqueued on
 * params->stream (0: the null stream) and not waited for.  The 1-D operators and the face
 * traces are kept in a static device array of 64 MiB per GPU, held from the library's load
 * until the process ends; the traces need nE * 2d * nvar * (N+1)^(d-1) * 8 bytes (twice
 * that with BR1) of it after 4 KiB for the operators, and larger meshes are refused with
 * HBPC_ERR_ARG before any device work.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other host threads) race and must be serialised
 * by the caller.  Errors (returned only, there is no context for hbpc_last_error):
 * HBPC_ERR_ARG, HBPC_ERR_UNSUPPORTED as for hbpc_create and for HBPC_EQ_NAVIER_STOKES (whose
 * BR2 face gradients are not kept in the scratch), HBPC_ERR_HIP. */
int hbpc_residual1_noalloc(const hbpc_mesh* mesh, int N, int equation, const hbpc_params* params,
                           const double* w, double* r1);
/* R2_h(w, sigma) = R1_h'(w) sigma -> r2 (Eq. DGSEM_wtt, exact directional
 * derivative).  sigma == NULL: sigma = R1_h(w) is computed first. */
int hbpc_residual2(hbpc_ctx* ctx, const double* w, const double* sigma, double* r2);
/* Extended residual of Sec. 3.2.1 with X = (w, sigma):
 *   G[0:ndof]      = w - a1dt R1(w) + bcoef R2(w, sigma) - b
 *   G[ndof:2ndof]  = sigma - R1(w)
 * a1dt = alpha_1 dt, bcoef = alpha_2 dt^2 / 2 (Eq. Newton_Residual). */
int hbpc_newton_residual(hbpc_ctx* ctx, const double* w, const double* sigma, const double* b,
                         double a1dt, double bcoef, double* G);
/* Extended Jacobian-vector product (Eq. nonlinear_eqsys):
 *   JdX = ( dw - a1dt T1 + bcoef (T2 + T3),  dsigma - T1 )
 *   T1 = R1'(w) dw, T2 = R1'(w) dsigma, T3 = R1''(w)[sigma, dw] (0 if params.hessian == 0)
 * dX and JdX hold 2 ndof values.  mode: HBPC_JVP_LINEARISED or HBPC_JVP_FD
 * (Eq. MatrixFree_nonlinear with eps_FD = sqrt(eps_mach)/(eps ||d||_2)). */
int hbpc_jvp(hbpc_ctx* ctx, const double* w, const double* sigma, double a1dt, double bcoef,
             const double* dX, double* JdX, int mode);
/* Same, linearised, in FP32 on FP32 copies of w and sigma. */
int hbpc_jvp_f32(hbpc_ctx* ctx, const float* w, const float* sigma, double a1dt, double bcoef,
                 const float* dX, float* JdX);

/* Build BJ_ext at state w (Sec. 3.2.3): K_i = element-local dR1/dw (every
 * quantity read from a neighbour held constant), S_i = I - a1dt K_i +
 * bcoef K_i^2, S_i^-1 by Gauss-Jordan elimination with partial pivoting
 * (element blocks of up to 1024 unknowns; HBPC_ERR_UNSUPPORTED above).  precision HBPC_FP64 or
 * HBPC_MIXED selects the storage (and arithmetic) of S^-1.  The blocks are
 * kept in the context until the next build (they share storage with the
 * first stage's blocks of hbpc_step). */
int hbpc_pc_build(hbpc_ctx* ctx, const double* w, double a1dt, double bcoef, int precision);
/* Build BJ^H_ext at the state (w, sigma) (Sec. 3.2.3): in addition to K_i,
 * H_i = element-local dR2/dw at (w, sigma), i.e. R1''(w)[sigma, .] with the
 * neighbours' sigma read and their w held constant; S_i = I - a1dt K_i +
 * bcoef (K_i^2 + H_i).  S_i no longer commutes with K_i, and the apply is
 * y = S_i^-1 (vw - bcoef K_i vs), P^-1 (vw, vs) = (y, vs + K_i y).  w and
 * sigma: ndof device values each, read only.  Same storage, limits and
 * precision rule as hbpc_pc_build; HBPC_ERR_ARG on a context whose params.precond
 * is HBPC_PC_LEARNED.  hbpc_pc_apply* below use whichever build came last. */
int hbpc_pc_build_hess(hbpc_ctx* ctx, const double* w, const double* sigma, double a1dt, double bcoef,
                       int precision);
/* With params.precond == HBPC_PC_LEARNED the build only records w (and its
 * FP32 copy for HBPC_MIXED) and the coefficients; apply then runs the learned
 * preconditioner (below) in FP64 or FP32 vectors.
 * Y = P^-1 X with the blocks of the last build: (D vw + E vs, F vw + G vs). */
int hbpc_pc_apply(hbpc_ctx* ctx, const double* X, double* Y);
int hbpc_pc_apply_f32(hbpc_ctx* ctx, const float* X, float* Y);

/* ----------------------------------------------------------------------
 * Learned preconditioner (an addition to the paper's method).
 *
 * It keeps the structure of BJ_ext (Sec. 3.2.3), the exact inverse of the
 * extended Jacobian of Eq. nonlinear_eqsys with R1'(w) replaced by its
 * element-local part K, and replaces the element solve S_e^-1,
 * S_e = I - a1dt K_e + bcoef K_e^2, by a network on patch features:
 *     rt = vw - bcoef K vs,
 *     dw_e = s_e f(x_e)             for every element e,
 *     ds = vs + K dw,
 * where f is a per-element network with two hidden layers of width H = 256
 * and ne = hbpc_block_size outputs, on the features x_e = [x_r | x_w] of
 * element e:
 *     x_r = rt tiles of (e, its 2d face neighbours in the order -x,+x,-y,+y,-z,+z) / s_e,
 *     x_w = [w tiles of the same elements, ln a1dt, ln bcoef],
 *     n_r = (2d+1) ne residual inputs, n_w = n_r + 2 state inputs, n_in = n_r + n_w,
 * each tile in the w[e][v][node] layout, s_e = RMS of the rt tiles + 1e-30.
 * The state path gates a residual path that is linear, so that for a fixed
 * state the preconditioner is a linear map of (vw, vs):
 *     g1 = relu(x_w W1w + b1),   g2 = relu(g1 W2w + b2),
 *     h1 = (x_r W1r) .* g1,      h2 = (h1 W2r) .* g2,      f = h2 W3.
 * Parameters theta (FP32), row-major, W[i][j] from input i to output j:
 * W1r (n_r x H), W1w (n_w x H), b1 (H), W2r (H x H), W2w (H x H), b2 (H),
 * W3 (H x ne).  The gates are computed once per linearisation state (per
 * Newton iteration, or per hbpc_pc_build), the residual path per apply.
 * Training: pairs collected by hbpc_step (hbpc_mlp_collect: Newton
 * corrections, or the element solves of BJ_ext on Krylov vectors), mean
 * squared error, Adam with FP32 master weights.
 * -------------------------------------------------------------------- */
/* Network shape of this context; any output pointer may be NULL. */
int hbpc_mlp_shape(const hbpc_ctx* ctx, int* n_in, int* hidden, int* n_out, size_t* n_params);
/* Load / read the FP32 parameter vector (device, n_params values).  Loading
 * resets the Adam moments and step count. */
int hbpc_mlp_set_params(hbpc_ctx* ctx, const float* theta);
int hbpc_mlp_get_params(hbpc_ctx* ctx, float* theta);
/* Seeded initial parameters: weights uniform in +-sqrt(g / fan_in), g = 6 on
 * the ReLU state path (W1w, W2w) and 3 on the linear residual path (W1r,
 * W2r, W3), from splitmix64 counters; zero biases; Adam state reset. */
int hbpc_mlp_init(hbpc_ctx* ctx, unsigned long long seed);
/* Feature rows of `count` elements: elems (device int array, or NULL for
 * elements 0..count-1; an entry outside 0..n_elem-1 gives a zero row and
 * scale 0), rt and w FP64 (ndof).  X: count x n_in FP32 out;
 * scale: count FP32 out (may be NULL); if dw != NULL, T: count x ne FP32 out
 * with T[r] = dw_e / s_e. */
int hbpc_mlp_features(hbpc_ctx* ctx, const double* rt, const double* w, const double* dw,
                      const int* elems, int count, double a1dt, double bcoef,
                      float* X, float* T, float* scale);
/* Network output Y (rows x ne) of feature rows X (rows x n_in, the layout
 * of hbpc_mlp_features); precision HBPC_MLP_*. */
int hbpc_mlp_forward(hbpc_ctx* ctx, const float* X, int rows, float* Y, int precision);
/* Mean squared error over rows x ne of f(X) - T and its gradient (device,
 * n_params FP32); the loss goes to *loss_host (synchronises). */
int hbpc_mlp_loss_grad(hbpc_ctx* ctx, const float* X, const float* T, int rows, float* grad,
                       double* loss_host, int precision);
/* One Adam step on the context's parameters with gradient grad (device):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, theta -= lr (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps). */
int hbpc_mlp_adam(hbpc_ctx* ctx, const float* grad, double lr, double beta1, double beta2, double eps);
/* Start collecting training pairs into caller-owned device buffers X
 * (capacity x n_in) and T (capacity x ne) during subsequent hbpc_step calls,
 * until capacity is reached; per_event distinct elements (drawn with
 * splitmix64 from seed) contribute one pair each per event:
 *   HBPC_MLP_PAIRS_NEWTON: event = every Newton correction dX of -G;
 *     features of rt = -G_w + bcoef K G_sigma, target = dw_e / s_e;
 *   HBPC_MLP_PAIRS_KRYLOV: event = every `every`-th FGMRES iteration of a
 *     BJ_ext solve; features of rt = vw - bcoef K vs of the Krylov vector v,
 *     target = the w block of BJ_ext's output for v (S_e^-1 rt_e) / s_e;
 *   HBPC_MLP_PAIRS_RANDOM: event = every `every`-th FGMRES iteration of
 *     any solve without the learned preconditioner; target dw = independent
 *     standard normal values (splitmix64 counters, Box-Muller), features of
 *     rt = dw - a1dt K dw + bcoef K (K dw), i.e. BJ_ext's element operator
 *     S_e applied exactly, target dw_e / s_e.
 * Each call restarts the count at 0 (pass offset pointers to append).
 * capacity 0 stops collecting.  hbpc_mlp_collected returns the pairs
 * written so far. */
#define HBPC_MLP_PAIRS_NEWTON 0
#define HBPC_MLP_PAIRS_KRYLOV 1
#define HBPC_MLP_PAIRS_RANDOM 2
int hbpc_mlp_collect(hbpc_ctx* ctx, float* X, float* T, size_t capacity, int per_event,
                     unsigned long long seed, int source, int every);
size_t hbpc_mlp_collected(const hbpc_ctx* ctx);

typedef struct {
    int epochs;                /* passes over the pairs */
    int batch;                 /* pairs per Adam step, 1..8192 */
    double lr, beta1, beta2, eps;  /* Adam */
    unsigned long long seed;   /* pair order per epoch: Fisher-Yates driven by splitmix64 */
    int precision;             /* HBPC_MLP_* */
} hbpc_train_cfg;
typedef struct {
    int steps;                 /* Adam steps taken */
    double loss_first;         /* mean loss over the first epoch's batches */
    double loss_last;          /* mean loss over the last epoch's batches */
    double ms;                 /* wall time */
} hbpc_train_log;
/* Defaults: 40 epochs, batch 256, lr 1e-3, (0.9, 0.999, 1e-8), seed 2109, BF16. */
void hbpc_default_train_cfg(hbpc_train_cfg* cfg);
/* Train the context's network on `count` pairs (X, T device, as collected).
 * Synchronises; log may be NULL. */
int hbpc_train_mlp(hbpc_ctx* ctx, const float* X, const float* T, size_t count,
                   const hbpc_train_cfg* cfg, hbpc_train_log* log);

/* One HBPC(q, k_max) step (Algorithm 1) of size dt, in place.  Transactional:
 * on any error w_inout is unchanged.  stats may be NULL.  Synchronises. */
int hbpc_step(hbpc_ctx* ctx, double* w_inout, double dt, hbpc_stats* stats);

/* Kernel timing (HIP events recorded around every launch on the context's
 * stream, resolved after synchronisation).  Classes: trace, r1, r2, res, jvp,
 * kcol, pcpre, bj_apply, bj_invert, mdot, gemv, vec, gs_dot, gs_update, lin
 * (x + c R1'(w) s), mlp_feat, mlp_gemm, mlp_vec, ns_grad (BR2 face gradients),
 * bj_apply4 (the apply to the four right-hand sides of two paired stage
 * systems, HBPC_PC_PAIRED).  `bytes` and `flops` are
 * the algorithmic figures of all recorded launches: inputs read once and
 * outputs written once (bytes), the method's floating-point operations
 * (flops, only for bj_invert and mlp_gemm).  Timing adds a few microseconds per launch. */
typedef struct {
    char name[16];
    int launches;
    double total_ms;
    double bytes;
    double flops;
} hbpc_kernel_prof;
int hbpc_profile_enable(hbpc_ctx* ctx, int enable);
/* Record only the launches of the named class (NULL: all classes again), to
 * time one kernel without the cost of events around every other launch.
 * Reset to all classes by hbpc_profile_enable.  HBPC_ERR_ARG for an unknown
 * name. */
int hbpc_profile_only(hbpc_ctx* ctx, const char* name);
/* Copy up to max classes (those with launches) into out; reset != 0 clears
 * the counters.  Synchronises the stream.  Returns the number of classes
 * written, or a negative error code. */
int hbpc_profile_read(hbpc_ctx* ctx, hbpc_kernel_prof* out, int max, int reset);

const char* hbpc_strerror(int code);
const char* hbpc_last_error(const hbpc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
