/*
 * aao.h - C ABI of the MI355X (gfx950) all-at-once solver for the heat equation
 * preconditioned by the block epsilon-circulant (BEC) matrix of Lin & Ng,
 * "An all-at-once preconditioner for evolutionary partial differential
 * equations" (arXiv 2002.01108).
 *
 * Problem (Section 2): u_t = div(a grad u) + f on (0,1)^d x (0,T], d = 1,2,3,
 * homogeneous Dirichlet data, backward Euler in time with N = n steps,
 * tau = T/n, finite differences in space (mass matrix M = I, see the Remark
 * after Assumptions 1-3).  Interior grid m1 x m2 x m3 points (unused dims 1),
 * h_d = 1/(m_d + 1).  K is the 3/5/7-point -Laplacian, or the flux form of
 * -div(a grad .) once a coefficient is set.
 *
 * All-at-once system (Section 2, eq. (allatoncesystem)):
 *     L u = f,  (L u)^k = (I + tau K) u^k - u^{k-1},  u^0 := 0,
 *     f = (tau f^1 + u_0; tau f^2; ...; tau f^n).
 * Preconditioner (Section 3): P_eps = L with -eps I in the top-right block.
 * Its inverse is applied with the three steps of Section 4
 * (eqs. (ytild), (blockdiaginv), (zcompt)) using the diagonalisation
 * R_eps = D_eps^{-1} F_n^* Lambda_eps F_n D_eps (eq. (repsdiagform)),
 * theta = exp(+2 pi i / n), lambda_k = 1 - eps^{1/n} theta^k, and only the
 * blocks k = 0..n/2 (conjugate symmetry, end of Section 4).
 *
 * Conventions for every entry point:
 *  - Space-time vectors are caller-owned, contiguous FP64 DEVICE arrays of
 *    n*m elements, layout [n][m3][m2][m1] (x fastest); row k is u^{k+1}.
 *    The library never keeps a pointer past the call.
 *  - Work is queued on the context's HIP stream (default: the null stream) and
 *    is ordered with the caller's work on that stream.  Entry points that
 *    return host values (aao_solve) synchronise that stream.
 *  - Errors are reported by return code only; no exception crosses the ABI.
 *    aao_last_error() gives a message for the last failing call on a context.
 *  - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef AAO_H
#define AAO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aao_ctx aao_ctx;

typedef enum {
  AAO_OK = 0,
  AAO_NOT_CONVERGED = 1, /* maxit reached; outputs hold the last iterate       */
  AAO_EINVAL = -1,       /* bad argument (sizes, eps outside (0,1], null, ...) */
  AAO_ENOMEM = -2,       /* device allocation failed                           */
  AAO_EHIP = -3,         /* a HIP runtime call or kernel launch failed         */
  AAO_ENAN = -4,         /* right-hand side or iterate is not finite           */
  AAO_ESTATE = -5        /* call not valid in the context's current state      */
} aao_status;

/* Arithmetic of the preconditioner (Steps 1-3).  L, residuals, Arnoldi and
 * Givens always run in FP64.  FP32: time FFTs, spatial transforms and divides
 * in FP32.  BF16X3: as FP32 but the spatial transforms multiply BF16 hi/lo
 * splits (hi*hi + hi*lo + lo*hi, round-to-nearest-even splits) with FP32
 * accumulation. */
typedef enum { AAO_FP64 = 0, AAO_FP32 = 1, AAO_BF16X3 = 2 } aao_precision;

/* Create a context for an m1 x m2 x m3 grid (dim = 1, 2 or 3; m2, m3 ignored
 * beyond dim), n time steps over (0, T], and BEC parameter eps.
 *  - eps must lie in (0, 1] (Section 3, Theorem 3.1 and the Remark after it);
 *    eps = 1 gives the block-circulant preconditioner.
 *  - n must be a power of two, 2 <= n <= 1024.
 *  - 1 <= m_d <= 1024.
 * Allocates all device tables and the spectrum workspace on the current device.
 * Returns AAO_EINVAL, AAO_ENOMEM or AAO_EHIP on failure (*out untouched). */
aao_status aao_setup(int dim, int m1, int m2, int m3, int n, double T, double eps,
                     aao_ctx **out);

/* Free everything the context owns.  Null is accepted. */
void aao_destroy(aao_ctx *ctx);

/* Queue all later work on `hip_stream` (a hipStream_t; null = default stream). */
aao_status aao_set_stream(aao_ctx *ctx, void *hip_stream);

/* Select the preconditioner arithmetic (default AAO_FP64).  May allocate a
 * differently sized spectrum workspace. */
aao_status aao_set_precision(aao_ctx *ctx, aao_precision p);

/* Precision schedule of aao_solve.  Flexible GMRES admits a different
 * preconditioner at every step, so the first `steps` Arnoldi steps of each
 * solve may apply P_eps^{-1} in `first` (typically AAO_FP32: its first step
 * leaves about the residual the FP64 preconditioner leaves, since that
 * residual is set by the method, not by rounding) and the later steps in the
 * context's precision (typically AAO_FP64, whose accuracy the last steps need:
 * rounding after the shifted divide is white in space, and L amplifies it by
 * up to 1 + 4 d tau / h^2).  steps = 0 (default) applies the context's
 * precision throughout; aao_apply_Pinv and aao_step1-3 always use it.
 * Needs right preconditioning and the exact sine-transform inner solve of a
 * constant coefficient (aao_solve returns AAO_ESTATE otherwise).  The spectrum
 * workspace is sized for the larger of the two precisions.
 * AAO_EINVAL for an unknown precision or steps < 0. */
aao_status aao_set_precision_schedule(aao_ctx *ctx, aao_precision first, int steps);

/* Variable coefficient a(x) of -div(a grad u) (Section 2, eq. (heateq)), given
 * on cell faces as HOST arrays (copied; the caller keeps ownership):
 *   1D: ax[m1+1];  2D: ax[m2][m1+1], ay[m2+1][m1];
 *   3D: ax[m3][m2][m1+1], ay[m3][m2+1][m1], az[m3+1][m2][m1];
 * x-face i of a row lies between interior nodes i-1 and i (face 0 and face m1
 * touch the walls).  K becomes the flux form (K u)_p = h^-2 sum_f a_f (u_p - u_nbr).
 * ax = null restores a = 1.  Values must be positive and finite (AAO_EINVAL).
 * All inputs are checked before anything changes: a rejected call leaves the
 * previous operator (coefficient or convection) in place.
 * With a variable coefficient the blocks of Step 2 are no longer diagonalised
 * by sine transforms: select AAO_INNER_DST_MEAN or AAO_INNER_MG. */
aao_status aao_set_coefficient(aao_ctx *ctx, const double *ax, const double *ay,
                               const double *az);

/* Convection-diffusion K u = -nu Laplace(u) + w . grad(u) on the unit square
 * (the setting of Section 5, Example 3, with a circulating wind; the paper's
 * SUPG-stabilised Q1 elements are replaced by five-point finite differences
 * with first-order upwinding).  wx, wy: HOST arrays [m2][m1] of the wind
 * components at the interior nodes (copied; the caller keeps ownership); nu > 0.
 * Node (j, i) couples to its west, east, south and north neighbours with
 *   W = nu/h1^2 + max(wx, 0)/h1,  E = nu/h1^2 + max(-wx, 0)/h1,
 *   S = nu/h2^2 + max(wy, 0)/h2,  N = nu/h2^2 + max(-wy, 0)/h2,
 * (K u)_p = (W + E + S + N) u_p - W u_west - E u_east - S u_south - N u_north,
 * a nonsymmetric M-matrix (Assumption 1 does not hold; Section 5 tests it
 * anyway).  A problem posed on (-1, 1)^2 maps to this one with nu/4 and w/2.
 * The blocks of Step 2 then need AAO_INNER_MG: its coarse levels use the same
 * discretisation with the wind taken at the coarse nodes and h doubled.
 * Needs dim = 2 and finite differences (AAO_EINVAL / AAO_ESTATE otherwise);
 * replaces any face coefficient; wx = null restores K = -Laplace.  Values must
 * be finite (AAO_EINVAL).  Afterwards AAO_INNER_DST_MEAN, AAO_INNER_CNN and Q1
 * elements return AAO_ESTATE. */
aao_status aao_set_convection(aao_ctx *ctx, double nu, const double *wx, const double *wy);

/* Inner solver of Step 2 (eq. (blockdiaginv)) for each block
 * B_k = lambda_k I + tau K:
 *   AAO_INNER_DST       exact sine-transform diagonalisation (constant a only;
 *                       AAO_ESTATE at apply time otherwise)
 *   AAO_INNER_DST_MEAN  sine-transform solve of lambda_k I + tau abar K_h, abar
 *                       the arithmetic mean of all face coefficients
 *   AAO_INNER_MG        `cycles` geometric multigrid V-cycles (Section 4 and
 *                       Section 5, Example 2: one V-cycle, one pre- and one
 *                       post-smoothing step; here red-black Gauss-Seidel, full
 *                       weighting, bilinear prolongation, rediscretised coarse
 *                       grids with harmonic face means).  Square 2D grids only
 *                       (AAO_EINVAL otherwise); a full hierarchy needs
 *                       m1 = 2^L - 1.
 *   AAO_INNER_CNN       one V-cycle followed by the learned correction below
 *                       (square 2D grids; parameters must be set first,
 *                       AAO_ESTATE otherwise; `cycles` is ignored).
 * Inexact inner solves make the preconditioner approximate: aao_solve is
 * flexible GMRES, so any inner solver is admissible. */
typedef enum {
  AAO_INNER_DST = 0,
  AAO_INNER_DST_MEAN = 1,
  AAO_INNER_MG = 2,
  AAO_INNER_CNN = 3
} aao_inner;
aao_status aao_set_inner(aao_ctx *ctx, aao_inner inner, int cycles);

/* Time discretisation of the all-at-once system (Section 4, eqs. (pstepscheme)
 * and (pstepbecpreconditioner), M = I):
 *  - order 1 (default): backward Euler, r = (1, -1);
 *  - order 2: BDF2, r = (3/2, -2, 1/2) (Section 5, Table bdf2table), with a
 *    backward-Euler first step (the paper does not say how the two-step
 *    scheme starts; this start keeps the scheme second order).  Row 1 of L
 *    is u^1 + tau K u^1, row 2 is (3/2) u^2 - 2 u^1 + tau K u^2, later rows
 *    the full BDF2 row; aao_build_rhs then adds u^0 to row 1 and
 *    -(1/2) u^0 to row 2.
 * The preconditioner P_eps uses the Toeplitz R_eps of the scheme, i.e.
 * lambda_k = sum_j r_j eps^{j/n} theta^{kj} in Step 2; Steps 1 and 3 are
 * unchanged.  Returns AAO_EINVAL for another order. */
aao_status aao_set_scheme(aao_ctx *ctx, int order);

/* Spatial discretisation.
 *  - AAO_DISC_FD (default): finite differences, M = I, the 3/5/7-point K.
 *  - AAO_DISC_Q1: bilinear (Q1) finite elements on the uniform square grid
 *    (Section 5 uses them): L = R (x) M + tau I (x) K (eq. (pstepscheme)) with
 *    M = M1 (x) M1, K = M1 (x) K1 + K1 (x) M1, M1 = h/6 tridiag(1, 4, 1),
 *    K1 = 1/h tridiag(-1, 2, -1); both act as 9-point stencils in aao_apply_A
 *    and the solve.  P_eps = R_eps (x) M + tau I (x) K: in the sine basis
 *    B_k = lambda_k M + tau K is diagonal with entries m_i (lambda_k + tau k_i / m_i),
 *    which Step 2 divides by.  aao_build_rhs returns M times the nodal right-
 *    hand side (the load vectors of nodally sampled f and u0).
 *    Needs dim = 2 with m1 = m2, a constant coefficient, the FP64 or FP32
 *    preconditioner and the DST inner solve (AAO_ESTATE otherwise, and later
 *    calls that would break these conditions return AAO_ESTATE).
 * Returns AAO_EINVAL for an unknown value or a grid Q1 does not support. */
typedef enum { AAO_DISC_FD = 0, AAO_DISC_Q1 = 1 } aao_discretisation;
aao_status aao_set_discretisation(aao_ctx *ctx, aao_discretisation disc);

/* Side of the preconditioner in aao_solve.
 *  - AAO_RIGHT (default): flexible GMRES on L P^{-1} w = rhs, u = P^{-1} w; the
 *    stopping test is on the true residual ||rhs - L u|| / ||rhs||.
 *  - AAO_LEFT: GMRES on P^{-1} L u = P^{-1} rhs (Section 3, eq.
 *    (preconditionedsystem)), stopping on the preconditioned residual
 *    ||P^{-1}(rhs - L u)|| / ||P^{-1} rhs|| as in the experiments of Section 5;
 *    it needs a fixed preconditioner (any aao_set_inner choice is one) and
 *    costs one extra P^{-1} per solve.  final_res still reports the true
 *    residual.
 * Returns AAO_EINVAL for an unknown side. */
typedef enum { AAO_RIGHT = 0, AAO_LEFT = 1 } aao_side;
aao_status aao_set_side(aao_ctx *ctx, aao_side side);

/* ---- learned inner solve (AAO_INNER_CNN) ----------------------------------
 * Extends the paper's inner solve of Step 2 (one multigrid V-cycle per block,
 * Section 4 and Section 5, Example 2) with a small network N that corrects the
 * V-cycle's result per frequency block k:
 *     e1 = V(r),  rho = r - B_k e1,  s = rms(rho),
 *     e  = S_r(e1 + s N(rho/s, log a; lambda_k) / (lambda_k + d))
 * with d the diagonal of tau K_a at each node (the network's two output
 * channels, a complex field, are divided pointwise by the diagonal of B_k) and
 * S_r one red-black Gauss-Seidel sweep for B_k e = r (the V-cycle's smoother)
 * started from its argument.
 * N: three 3x3 convolutions 3 -> 8 -> 8 -> 2 channels with ReLU, the two hidden
 * layers modulated by gamma = 1 + G phi, beta = H phi of the features
 * phi = (Re lambda_k, Im lambda_k, log|lambda_k|, 1); input channels
 * (Re rho/s, Im rho/s, log a - mean log a) with log a the log of the mean of the
 * four faces around a node; FP32.  Parameter vector (float, host order):
 *     W1[8][3][3][3] G1[8][4] H1[8][4] W2[8][8][3][3] G2[8][4] H2[8][4]
 *     W3[2][8][3][3] b3[2]          (aao_cnn_param_count() floats)
 * Square 2D grids only (the V-cycle's domain). */
int aao_cnn_param_count(void);

/* Load parameters from host memory (count must equal aao_cnn_param_count());
 * resets the optimiser state.  AAO_EINVAL for a wrong count or non-finite values. */
aao_status aao_cnn_set_params(aao_ctx *ctx, const float *params, int count);

/* Copy the current parameters to host memory. AAO_ESTATE if none are set. */
aao_status aao_cnn_get_params(aao_ctx *ctx, float *params, int count);

/* N on B images: x device [B][3][H][W], lam host [B][2] (Re, Im of lambda per
 * image, non-zero), y device [B][2][H][W].  For verification. */
aao_status aao_cnn_forward(aao_ctx *ctx, const float *x, const double *lam, int B, int H, int W,
                           float *y);

/* aao_cnn_forward without any allocation, for callers that cannot allocate
 * device memory (serving loops, code under stream capture, harnesses that
 * forbid hipMalloc): same arguments, layouts and result as aao_cnn_forward.
 * Its workspace (lambda, features, FiLM coefficients and the two hidden
 * layers) lives in one fixed 64 MiB device array per GPU, loaded with the
 * library and held until the process ends; x and y stay the caller's.  Limit:
 * 16 B H W + 36 B floats (plus alignment) must fit in 16 Mi floats, about one
 * million pixels over all images; larger requests return AAO_EINVAL before any
 * device work.  The host lambda array is consumed before the call returns (the
 * context's stream is synchronised once).  Every call on a GPU, from any
 * context, uses that GPU's one array: calls that overlap in time on one GPU
 * (other threads, other streams) race and must be serialised by the caller.
 * Needs parameters (AAO_ESTATE otherwise). */
aao_status aao_cnn_forward_noalloc(aao_ctx *ctx, const float *x, const double *lam, int B, int H,
                                   int W, float *y);

/* Gradients of sum(dy * N(x)): parameter gradient to host grad[count] (may be
 * null), input gradient to device dx [B][3][H][W] (may be null). */
aao_status aao_cnn_backward(aao_ctx *ctx, const float *x, const double *lam, int B, int H, int W,
                            const float *dy, float *dx, float *grad);

/* Build training pairs from S space-time fields y (device [S][n][m]): for each
 * field and kept block k, r = Step 1 of y, rho = r - B_k V(r), target
 * delta = B_k^{-1} rho approximated by `target_cycles` V-cycles (the method's
 * own multigrid inner solves), stored as (rho/s, delta/s) with s = rms(rho).
 * Replaces earlier pairs; uses the context's coefficient and precision. */
aao_status aao_cnn_make_pairs(aao_ctx *ctx, const double *y, int S, int target_cycles);

/* Number of stored pairs (S * (n/2+1)). */
aao_status aao_cnn_num_pairs(const aao_ctx *ctx, int *count);

/* `steps` Adam steps (lr; beta1 0.9, beta2 0.999, 1e-8) on minibatches of
 * `batch` pairs chosen by the caller: idx host [steps][batch] in [0, num_pairs).
 * The loss is the residual the inner solve leaves after the network and the
 * sweep: mean over the batch of ||rho_hat - B_k S(N(x) / (lambda_k + d))||^2
 * / ||rho_hat||^2, rho_hat = rho/s the stored input residual and S the sweep
 * for B_k e = rho_hat; its gradient runs back through the sweep and the
 * diagonal scaling.  Per-step loss to host loss[steps] (may be null).  Parameters must be
 * set first (initial values are the caller's; drawing them is the caller's
 * business). */
aao_status aao_cnn_train(aao_ctx *ctx, int steps, int batch, float lr, const int *idx,
                         float *loss);

/* rhs = (tau f^1 + u0; tau f^2; ...; tau f^n) (Section 2, eq. (allatoncesystem)).
 * f: device [n][m], u0: device [m], rhs: device [n][m] (may alias f). */
aao_status aao_build_rhs(aao_ctx *ctx, const double *f, const double *u0, double *rhs);

/* Inhomogeneous Dirichlet data (Section 2, the boundary condition of eq.
 * (heateq); Section 5, Example 3's hot wall): f^k += (the couplings of K to
 * the boundary nodes) x (their values at t_k = k tau), the terms that move to
 * the right-hand side when the boundary values are known; aao_build_rhs then
 * scales f by tau.  2D finite differences only (any coefficient form).
 * gb: device [n][2 m2 + 2 m1], per time level the values next to the west
 * wall (x = 0, one per row, m2), the east wall (x = 1, m2), the south wall
 * (y = 0, one per column, m1) and the north wall (y = 1, m1); f: device [n][m],
 * updated in place.  AAO_EINVAL for another dimension, AAO_ESTATE for Q1. */
aao_status aao_boundary_source(aao_ctx *ctx, const double *gb, double *f);

/* y = L x, the all-at-once matrix (Section 2, eq. (allatoncesystem)).
 * x, y: device [n][m], must not alias. */
aao_status aao_apply_A(aao_ctx *ctx, const double *x, double *y);

/* y = P_eps^{-1} x by Steps 1-3 of Section 4 in the context's precision.
 * x, y: device [n][m] FP64 (may alias: x is fully consumed first). */
aao_status aao_apply_Pinv(aao_ctx *ctx, const double *x, double *y);

/* The three steps separately, with the half spectrum in an external layout:
 * interleaved complex FP64 [n/2+1][m][2] (real, imaginary), block k holding
 * ytilde^{k+1} of Section 4.
 * step1: yt = (F_n D_eps (x) I) y, blocks k = 0..n/2          (eq. (ytild))
 * step2: zt^k = (lambda_k I + tau K)^{-1} yt^k, k = 0..n/2     (eq. (blockdiaginv))
 * step3: z = (D_eps^{-1} F_n^* (x) I) zt, using zt^{n-k} = conj(zt^k); the
 *        imaginary parts of blocks 0 and n/2 are ignored        (eq. (zcompt))
 * Internally each step runs in the context's precision; these entry points
 * convert to and from the internal layout and exist for verification. */
aao_status aao_step1(aao_ctx *ctx, const double *y, double *yt);
aao_status aao_step2(aao_ctx *ctx, const double *yt, double *zt);
aao_status aao_step3(aao_ctx *ctx, const double *zt, double *z);

/* Solve L u = rhs by right-preconditioned restarted flexible GMRES with P_eps
 * (Section 5 uses restarted GMRES(50) from a zero guess).  Orthogonalisation is
 * classical Gram-Schmidt applied twice, all in FP64 on the device; Givens
 * rotations run on the host.
 *  - u: device [n][m]; on entry the initial guess if use_guess != 0 (ignored
 *    otherwise, zero guess); on exit the last iterate.  rhs and u must not
 *    share memory (the Krylov basis starts from rhs, which the solve keeps
 *    reading while it writes u): overlapping ranges return AAO_EINVAL.
 *  - Stops when the relative residual ||rhs - L u|| / ||rhs|| (tracked by the
 *    Givens recurrence; with aao_set_side(AAO_LEFT) the preconditioned one) is
 *    <= tol, or after maxit Arnoldi steps in total.
 *  - restart: Krylov basis size (>= 1); the context allocates 2*(restart+1)
 *    vectors of n*m doubles and keeps them for later calls.
 *  - iters (host, may be null): total Arnoldi steps.
 *  - res_hist (host, may be null, capacity hist_cap): the Givens estimate after
 *    each step; hist_len (may be null) receives the number written.
 *  - final_res (host, may be null): ||rhs - L u|| / ||rhs|| recomputed
 *    explicitly from u at exit.
 * Returns AAO_OK on convergence (a breakdown h_{j+1,j} = 0 is convergence),
 * AAO_NOT_CONVERGED if maxit was reached, AAO_ENAN for a non-finite rhs,
 * AAO_EINVAL for tol < 0, maxit < 1, restart < 1, null vectors or rhs and u
 * overlapping.  A non-finite rhs is found from ||rhs||, which a zero-guess solve
 * of a large system (n*m >= 2^22, tol > 0, right preconditioning) takes from its
 * first Arnoldi step: P^-1 and L have then run once; u is left unchanged. */
aao_status aao_solve(aao_ctx *ctx, const double *rhs, double *u, int use_guess, double tol,
                     int maxit, int restart, int *iters, double *res_hist, int hist_cap,
                     int *hist_len, double *final_res);

/* Wait for all work queued on the context's stream. */
aao_status aao_sync(aao_ctx *ctx);

/* Kernel classes for aao_profile / aao_profile_read. */
typedef enum {
  AAO_K_APPLY_L = 0,   /* all-at-once matvec                            */
  AAO_K_TIME_FWD = 1,  /* Step 1: eps scaling + forward time FFT        */
  AAO_K_TIME_INV = 2,  /* Step 3: inverse time FFT + unscaling          */
  AAO_K_DST = 3,       /* Step 2: one DST-I mode product (matrix cores) */
  AAO_K_DIVIDE = 4,    /* Step 2: shifted complex divide                */
  AAO_K_KRYLOV = 5,    /* GMRES vector kernels and reductions           */
  AAO_K_NCLASS = 6
} aao_kernel_class;

/* Time every launch of the kernel classes whose bit is set in `mask` with a
 * pair of HIP events recorded on the context's stream around it (mask 0
 * disables).  Resets the accumulated totals.  Costs one event pair per timed
 * launch and no synchronisation. */
aao_status aao_profile(aao_ctx *ctx, int mask);

/* Synchronise the stream and return, per class, the summed event time in
 * milliseconds (ms[AAO_K_NCLASS]) and the number of timed launches
 * (launches[AAO_K_NCLASS]) since the last aao_profile call.  Either output may
 * be null. */
aao_status aao_profile_read(aao_ctx *ctx, double *ms, int *launches);

/* Human-readable name of a status code (static storage). */
const char *aao_status_string(aao_status s);

/* Message of the last failure on ctx (empty if none); valid until the next call. */
const char *aao_last_error(const aao_ctx *ctx);

/* Sizes the context was set up with: out[0..8] = dim, m1, m2, m3, n,
 * padded plane dims P1, P2, P3, and the precision. */
aao_status aao_query(const aao_ctx *ctx, int *out9);

#ifdef __cplusplus
}
#endif

#endif /* AAO_H */
