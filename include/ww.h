/*
 * ww.h -- C ABI of the MI355X (gfx950) engine for the Dirichlet-Neumann / Jacobian hot
 * path of the overdetermined shooting method for standing water waves
 * (Wilkening & Yu, "Overdetermined shooting methods for computing standing water waves
 * with spectral accuracy").
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - Grid: alpha_j = 2 pi j / N, j = 0..N-1 (uniform mesh, x = alpha); N even, of the
 *    form 2^a 3^b, 16 <= N <= n_max <= 2048.
 *  - Surface: `surface` / eta is the displacement from the still level.  At finite
 *    mean depth h the surface height is h + eta and the bottom is y = 0 (App. A);
 *    h = INFINITY (or h <= 0) selects infinite depth.
 *  - Arrays are column-major doubles.  A state vector is 2N doubles [eta | phi].
 *  - Pointers marked "device" are device memory of the GPU current when the context
 *    was created; "host" pointers are host memory.  The caller owns every array it
 *    passes; the library keeps no caller pointer after a call returns, except the
 *    stream.  Input and output arrays must not alias.
 *  - All GPU work is enqueued on the context's stream (the caller's, normally torch's
 *    current stream).  Calls that return a host scalar (f, df/dT) or report a device
 *    status (pivot guard, non-finite state) synchronise that stream; the others are
 *    stream-ordered.
 *  - Return value: 0 on success, a negative WW_E* code otherwise; ww_last_error()
 *    returns a thread-local message for the last failure.
 */
#ifndef WW_H
#define WW_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ww_ctx ww_ctx;

/* status codes */
#define WW_OK 0
#define WW_EINVAL (-1)     /* bad argument: null pointer, N not even / not 2^a 3^b / > n_max,
                              nrhs or M too large, non-explicit tableau */
#define WW_ENOSETUP (-2)   /* dtn_solve_multi before dtn_setup, shoot_* before shoot_setup */
#define WW_EHIP (-3)       /* HIP runtime failure; the message carries the HIP error string */
#define WW_EDOMAIN (-4)    /* finite depth with surface height h + eta <= 0 somewhere */
#define WW_ENONFINITE (-5) /* NaN or Inf in the marched state */
#define WW_EPIVOT (-6)     /* a pivot fell below the guard: of the unpivoted LU in a
                              WW_STRICT context, else of the partially pivoted fallback
                              (A numerically singular) */
#define WW_EREFINE (-7)    /* mixed precision, WW_STRICT context: refinement did not reach
                              its tolerance (without WW_STRICT the FP64 fallback runs) */
#define WW_ENOCONV (-8)    /* an iteration did not converge (thin SVD) */

/* context flags */
#define WW_FP64 0u         /* LU, triangular solves, everything in FP64 */
#define WW_MIXED 1u        /* LU and triangular solves in FP32 on MFMA, FP64 iterative
                              refinement of every solve (residuals in FP64): a fixed number
                              of sweeps (2; environment WW_NREF, 0..8; 0 leaves the FP32
                              solve, which then fails the test), then the FP64
                              residual of the final solution must be at most 2^-43 of
                              the right-hand side in every column (max norm), else
                              the call is redone with FP64 factors (WW_FB_FP64), or
                              fails with WW_EREFINE in a WW_STRICT context */
#define WW_STRICT 2u       /* no fallbacks: report WW_EPIVOT / WW_EREFINE instead */
#define WW_GMRES 4u        /* marches without Jacobian columns (shoot_eval with J = NULL,
                              the residual evaluations of ww_levmar) solve eq. (fred) for
                              the base state by GMRES (Sec. 2.2) instead of an LU: one cycle
                              of Arnoldi steps with classical Gram-Schmidt twice, stopping
                              when the residual estimate is below 1e-15 ||psi||; the step
                              budget is the count one solve of a rough right-hand side
                              takes on the initial surface, plus 4 (at most 32; environment
                              WW_GMRES_ITERS, 2..32, fixes it instead); the FP64 residual
                              must then pass the test of WW_MIXED, else the march is redone
                              with LU factors (WW_FB_DIRECT) */

/*
 * Fallbacks.  The block LU of A runs without row interchanges (A = I/2 + K/N is
 * diagonally dominant for graph surfaces; Sec. 3.3 does not discuss pivoting) behind a
 * guard on its pivots: every pivot must be at least 1e-8 in magnitude (environment
 * WW_PIVOT_GUARD, read by ww_create, replaces that bound for the unpivoted LU only; a
 * test hook for the fallback path).  When a pivot falls below the guard, the call is
 * redone with partial pivoting: Gaussian elimination with row interchanges (largest
 * magnitude in the column) fixes a row order P on the GPU, the block LU factors P A in
 * FP64, and every solve gathers its right-hand side by P (the adjoint scatters its
 * transposed solve by P^T).  A march is redone whole, without a step graph, on one
 * stream.  If a pivot of the pivoted factorisation is also below 1e-8 the call fails
 * with WW_EPIVOT.
 */
#define WW_FB_PIVOTED 1u   /* the results come from partially pivoted FP64 factors */
#define WW_FB_FP64 2u      /* the results come from FP64 factors after the mixed-precision
                              refinement test failed */
#define WW_FB_DIRECT 4u    /* the lagged-factor solves of a single-instance march (see
                              shoot_eval), or the GMRES solves (WW_GMRES), failed their
                              residual test; the march was redone with every stage's own
                              LU factors, in the context's precision form */

/*
 * ww_create: allocate a context whose device workspace serves every N <= n_max and
 * every right-hand-side count (M + 1) <= r_max.  `hip_stream` is a hipStream_t (NULL:
 * the default stream).  The library owns the workspace until ww_destroy.
 * The default time-stepping tableau is unset: ww_set_tableau must be called before
 * shoot_eval / shoot_adjoint (the Python layer loads DOP853).
 */
int ww_create(ww_ctx **ctx, int n_max, int r_max, unsigned flags, void *hip_stream);
void ww_destroy(ww_ctx *ctx);
int ww_set_stream(ww_ctx *ctx, void *hip_stream);

/*
 * ww_set_tableau: explicit Runge-Kutta tableau used for the march (Sec. 2.2 uses the
 * 12 stages of DOP853 for the 8th-order update).  a: s x s row-major (host), strictly
 * lower triangular; b: s weights (host); c: s nodes (host, unused: the system is
 * autonomous).  1 <= s <= 16.  Errors: WW_EINVAL if a is not strictly lower triangular.
 */
int ww_set_tableau(ww_ctx *ctx, int s, const double *a, const double *b, const double *c);

/*
 * dtn_setup (Sec. 2.1 eq. (fred), Sec. 2.2 eq. (K1K2), App. A): for the surface
 * `surface` (device, N), assemble the collocation matrices A = I/2 + K/N and
 * Gm = G/N of the second-kind boundary integral equation and of the normal-derivative
 * formula, and factor A once (LU, Sec. 3.3).  `tau` is stored for reference only (it
 * does not enter A or Gm).  Synchronises to check the pivot guard; a pivot below it
 * refactors with partial pivoting (WW_FB_PIVOTED).  The factors serve dtn_solve_multi
 * until the next dtn_setup, shoot_setup, shoot_eval or shoot_adjoint on the context.
 * Errors: WW_EINVAL, WW_EDOMAIN (finite depth, h + eta <= 0), WW_EPIVOT, WW_EHIP.
 */
int dtn_setup(ww_ctx *ctx, const double *surface, double h, double tau, int N);

/*
 * dtn_solve_multi (eq. (fred), (G)): for each of the nrhs columns psi of `rhs`
 * (device, N x nrhs, ld N) solve A mu = psi with the factors of the last dtn_setup,
 * form gamma = d mu / d alpha and return the Dirichlet-Neumann output
 * G psi = (1/2) H gamma + Gm gamma in `dtn_out` (device, N x nrhs, ld N).  `mu_out`
 * (device, N x nrhs, or NULL) receives mu.  nrhs <= r_max.  Stream-ordered, except in a
 * WW_MIXED context, where it synchronises to check the refinement test; a failed test
 * refactors A in FP64 (kept for later calls) and solves again (WW_FB_FP64).
 * Errors: WW_ENOSETUP, WW_EINVAL, WW_EPIVOT, WW_EREFINE (WW_STRICT), WW_EHIP.
 */
int dtn_solve_multi(ww_ctx *ctx, const double *rhs, int nrhs, double *dtn_out, double *mu_out);

/*
 * dtn_solve_multi_noalloc: dtn_solve_multi for callers that cannot allocate device
 * memory -- code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  Same arguments, results and errors as dtn_solve_multi (with the factors
 * of the last dtn_setup on the context), but its per-call work arrays (the padded
 * right-hand sides, the intermediate solves, gamma, (1/2) H gamma, the DtN output and
 * the mixed-form residuals) live in one fixed device array of WW_SCRATCH_BYTES per GPU
 * instead of the context's workspace; the call itself allocates nothing.  Limit:
 * 7 Np nrhs doubles must fit that array (Np = N rounded up to 64; e.g. N = 1024 with
 * nrhs <= 585, N = 2048 with nrhs <= 292), else WW_EINVAL.  The results are those of
 * dtn_solve_multi, bit for bit (the same kernels in the same order).  Every call on a GPU uses
 * that GPU's one array, which keeps the last call's contents: calls that overlap on
 * one GPU (on different streams, or from different threads) race; calls ordered on
 * one stream do not.  The array is held until the process ends.
 */
#define WW_SCRATCH_BYTES (32u << 20)
int dtn_solve_multi_noalloc(ww_ctx *ctx, const double *rhs, int nrhs, double *dtn_out, double *mu_out);

/*
 * shoot_setup (Sec. 3.1 eq. (init:stand), Sec. 3.3 eq. (q:qdot)): define the initial
 * state q0(c) = q_fixed + basis c, c in R^M, and the Jacobian seeds Qdot(0) = basis.
 * basis: device, 2N x M, column k = (eta part; phi part).  q_fixed: device 2N or NULL
 * (zero).  g: gravity, tau: surface tension / density.  M + 1 <= r_max.  The arrays are
 * copied into the context.
 */
int shoot_setup(ww_ctx *ctx, int N, double h, double tau, double g, const double *basis,
                const double *q_fixed, int M);

/*
 * shoot_eval (Sec. 3.1 eq. (f:phi), Sec. 3.3 eq. (Jik), (q:qdot); Sec. 3.2 eq. (dfdT)):
 * march (q, Qdot) with `nsteps` fixed steps of the tableau, dt = T / (4 nsteps), to
 * T/4 (T is the full period), with the 36th-order filter on every right-hand side and
 * after every step.  Outputs (device, caller-owned):
 *   r    (N)      r_i = phi(alpha_i, T/4) / sqrt(N)
 *   J    (N x M)  J_ik = phidot_k(alpha_i, T/4) / sqrt(N), or NULL (base only, R = 1)
 *   drdT (N)      dr/dT = phi_t(alpha_i, T/4) / (4 sqrt(N)), or NULL
 *   f    (host)   f = r.r / 2, or NULL
 * Lagged factors (L = 8; environment WW_PIPE_LAG, 0..11, read by ww_create; 0 turns
 * them off): in a march of one instance, the base chain of stage s (the march's
 * critical path) solves with the explicit inverse of stage s - L (the first product in
 * the same launch as the assembly of its own matrix) and refines the solution with
 * the FP64 residual of its own matrix (the same number of sweeps and the same
 * convergence test as WW_MIXED; environment WW_NREF_LAG, 1..8, sets the sweeps of
 * these solves alone), while its own matrix is factored concurrently: the LUs of G
 * consecutive stages (G = 2, at most L; environment WW_LU_GROUP, 1..4) share one
 * launch sequence, on one of the context's LU streams (group g on stream g mod K,
 * K = 3; environment WW_LU_STREAMS, 1..L).  The column chain of stage s uses that
 * stage's own factors and runs on the LU stream of its group after the group's LU,
 * the column chains in stage order (WW_COLS_ON_LU=0: on a column stream of their own,
 * with K = 2).  Each branch of a stage (spectral prep and assembly; the LU of a group;
 * the lagged base solve to the base right-hand side; the column chain) is a graph of
 * its own, replayed on its stream with the dependencies as events; the step end of the
 * base column runs on the caller's stream, that of the Jacobian columns after the last
 * column chain, and the caller's stream joins the others before the outputs.  The
 * results do not depend on K or on where the column chains run.  A
 * failed test (checked after the first step, and at the end) redoes the march with
 * every stage's own factors (WW_FB_DIRECT); the context's later marches then start that
 * way, until the next shoot_setup (not with WW_STRICT, which reports every failure).
 * Marches with and without J (M > 0 or J NULL) both use lagged factors; without J, on
 * at most two of the LU streams.
 * Synchronises to check the status flags.  A pivot below the guard anywhere in the
 * march redoes it with partial pivoting; a failed refinement test (WW_MIXED) redoes it
 * with FP64 factors (see ww_fallbacks).
 * Errors: WW_ENOSETUP, WW_EINVAL, WW_EPIVOT, WW_ENONFINITE, WW_EREFINE (WW_STRICT), WW_EHIP.
 */
int shoot_eval(ww_ctx *ctx, const double *params, double T, int nsteps, double *r, double *J,
               double *drdT, double *f);

/*
 * shoot_eval_sdc: shoot_eval marched with the 15th-order spectral deferred correction
 * of Sec. 2.2 instead of DOP853: per step of dt = T / (4 nsteps), eight Radau IIa nodes
 * (zeros of P_8 - P_7 on (0, 1]), initial values at the nodes by classical RK4 from node
 * to node, ten Picard sweeps Y_m <- y_0 + dt sum_j S_mj F(Y_j) (S: integrals of the
 * nodes' Lagrange polynomials), and the final integration with the weights of the last
 * node: 113 right-hand-side evaluations per step (every stage on its own factors, the
 * Jacobian columns with the base state of the same stage), the filter after every step.
 * The scheme is explicit: dt must resolve the largest frequency the filter passes (with
 * surface tension that is far smaller than DOP853's step).  The eight nodes of each
 * correction sweep are factored together and the column chains run on a second stream
 * (results bitwise those of one stream, which a context created with WW_NO_OVERLAP=1
 * and the pivoted and GMRES forms use).  In that two-stream form the second and third
 * RK4 stages of each predictor interval solve their base equations with the interval's
 * first factors, refined against their own matrix to the 2^-43
 * test (a miss redoes the march on direct factors: WW_FB_DIRECT; environment
 * WW_SDC_LAG=0 turns this off); every stage still factors its own matrix for its
 * Jacobian columns.  Without columns, the sweeps after the first solve each node on the
 * factors the first sweep made for it, refined the same way.  Outputs, fallbacks and errors as shoot_eval;
 * a failure's location names the step (its stage field is 0).  Synchronises.  Work
 * arrays are allocated at the first call: 113 x 2 n_max r_max doubles of stage slopes,
 * 17 x 2 n_max r_max doubles of stage states, and eight factor sets of n_max^2 size.
 */
int shoot_eval_sdc(ww_ctx *ctx, const double *params, double T, int nsteps, double *r, double *J,
                   double *drdT, double *f);

/*
 * shoot_eval_sdc_dd: the base march (no Jacobian) in double-double with SDC15, the
 * march of the quadruple-precision workflow (Sec. 2.2 on SDC and quadruple precision,
 * Sec. 3.3): every stage state, right-hand side of eq. (ww) (velocities of eq.
 * (uv:from:G), tension, zero-mean projection), the filter of eq. (filter) and the step's
 * combinations in double-double (about 32 digits), the nodes and weights to the same
 * precision; the DtN of each stage is dtn_setup_dd / dtn_solve_multi_dd (double-double
 * assembly and residuals, refinement from FP64 factors, or FP32 factors in a WW_MIXED
 * context).  Its own grid: N a power of
 * two, 16 <= N <= min(n_max, 1024); depth h (INFINITY for infinite depth), tension tau,
 * gravity g.  q0_hi, q0_lo: the initial state [eta | phi], 2N doubles each on the
 * device (q0_lo may be NULL for zero).  T = T_hi + T_lo, the full period (the march
 * runs nsteps steps of T / (4 nsteps) to T/4).  Outputs (device): r = phi(T/4)/sqrt(N)
 * as r_hi + r_lo (N each), dr/dT likewise (drdT_hi and drdT_lo both NULL to skip it;
 * it costs one more right-hand side); f (host, 2 doubles: hi, lo) = r.r/2.  Errors:
 * WW_EINVAL (arguments), WW_EDOMAIN (a stage surface through the bottom), WW_EPIVOT,
 * WW_EREFINE (a stage's solve misses its 2^-96 residual test), WW_ENONFINITE; the tests
 * run on the device and are read once per step (the error names the step).
 * Synchronises once per step.  Replaces the context's FP64 DtN factors and grid (call
 * dtn_setup or shoot_setup again before their entry points).
 */
int shoot_eval_sdc_dd(ww_ctx *ctx, int N, double h, double tau, double g, const double *q0_hi,
                      const double *q0_lo, double T_hi, double T_lo, int nsteps, double *r_hi,
                      double *r_lo, double *drdT_hi, double *drdT_lo, double *f);

/*
 * Double-double DtN (the GPU part of the quadruple-precision workflow: Sec. 2.2 on
 * quadruple precision, Sec. 3.3; residuals in extended precision by matrix products,
 * corrections from double-precision factors).  Values are unevaluated sums hi + lo of two
 * doubles (about 32 digits); every array is passed as a hi plane and a lo plane.
 * dtn_setup_dd: the surface eta = surface_hi + surface_lo (device, N each; surface_lo
 * may be NULL for zero) at depth h (as dtn_setup; h is a double): eta', eta'' by
 * double-double FFTs, exp(+-height) in double-double, A = I/2 + K/N and Gm = G/N of
 * eq. (fred), (G), (K1K2) assembled in double-double from double-double circulant
 * tables, and the FP64 factors (block LU and explicit inverse) of the leading part of A
 * (in a WW_MIXED context: of its FP32 copy, on MFMA).
 * N must be a power of two, 16 <= N <= min(n_max, 1024).  The FP64 factors of an earlier
 * dtn_setup are replaced (dtn_solve_multi then needs a new dtn_setup).  Synchronises.
 * Errors: WW_EINVAL, WW_EDOMAIN (finite depth, h + eta <= 0), WW_ENONFINITE, WW_EPIVOT
 * (a pivot below the guard: there is no pivoted double-double form), WW_EHIP.
 */
int dtn_setup_dd(ww_ctx *ctx, const double *surface_hi, const double *surface_lo, double h, int N);

/*
 * dtn_solve_multi_dd: G psi for nrhs columns (rhs_hi/rhs_lo: N x nrhs column-major,
 * device; rhs_lo may be NULL) in double-double: mu = A^{-1} psi from the FP64 inverse,
 * then three refinement sweeps r = psi - A mu (double-double products), mu += A_hi^{-1} r
 * (a WW_MIXED context: the FP32 inverse and six sweeps);
 * gamma = mu' and H gamma / 2 by double-double FFTs; G psi = H gamma / 2 + Gm gamma.
 * out_hi/out_lo (N x nrhs, caller-owned), and mu_hi/mu_lo (both or neither). The call
 * synchronises and checks the final residual: max |r| <= 2^-96 max |psi|, else
 * WW_EREFINE.  Errors: WW_EINVAL (null, nrhs out of 1..r_max), WW_ENOSETUP, WW_EREFINE,
 * WW_EHIP.
 */
int dtn_solve_multi_dd(ww_ctx *ctx, const double *rhs_hi, const double *rhs_lo, int nrhs, double *out_hi,
                       double *out_lo, double *mu_hi, double *mu_lo);

/*
 * Time segments on non-uniform meshes (Sec. 2.2 eq. (xi), (rho:def)).  The march to T/4
 * is split into segments l = 0..nseg-1 of theta_l T / 4 each (the theta_l sum to 1),
 * segment l with its own grid of N_l points and nsteps_l steps of theta_l T / (4
 * nsteps_l), on the mesh x = xi_l(alpha), alpha_j = 2 pi j / N_l:
 *   E_l = xi_l' = 1 - P[A_l sin^4(alpha/2)]   (refine_at = WW_REFINE_PI: finest at x = pi)
 *   E_l = xi_l' = 1 - P[A_l cos^4(alpha/2)]   (refine_at = WW_REFINE_ZERO: finest at x = 0)
 *   A_l = 8 (1 - rho_l) / (5 + 3 rho_l),  rho_l = min E_l / max E_l in (0, 1] (1: uniform)
 * The state and the Jacobian columns hold values at x_j = xi_l(alpha_j).  On the mapped
 * grid the kernels use zeta = xi + i eta (zeta' = E + i eta_alpha), x-derivatives
 * (1/E) d/dalpha, the DtN output divided by E, and the zero-mean projection in x (the
 * E-weighted mean); the filter acts in alpha.  Between segments every state column is
 * carried to the next mesh by its trigonometric interpolant in alpha evaluated at
 * xi_l^{-1}(xi_{l+1}(alpha_j)).  Mesh rule: if rho_{l+1} < rho_l then
 * N_{l+1} / N_l >= (5 + 3 rho_l) / (5 + 3 rho_{l+1}).
 */
#define WW_REFINE_PI 0
#define WW_REFINE_ZERO 1
typedef struct ww_segment {
  int N;          /* grid points (even, 2^a 3^b, 16 <= N <= n_max) */
  int nsteps;     /* steps of the segment (>= 1) */
  double theta;   /* fraction of T/4 (> 0; the fractions sum to 1 within 1e-12) */
  double rho;     /* mesh ratio, 0 < rho <= 1 */
  int refine_at;  /* WW_REFINE_PI or WW_REFINE_ZERO */
} ww_segment;

/*
 * shoot_eval_segments: shoot_eval over the segments segs[0..nseg-1] (1 <= nseg <= 64;
 * host array).  segs[0].N must equal shoot_setup's N: the basis and q_fixed are values
 * on the first segment's mesh.  Outputs on the last segment's grid (N = segs[nseg-1].N;
 * device, caller-owned), with the weights w_i = sqrt(E_i / N) of the mesh spacing:
 *   r (N) = w varphi(T/4),  J (N x M) = w phidot(T/4) or NULL,
 *   drdT (N) = w varphi_t(T/4) / 4 or NULL,  f (host) = r.r / 2 or NULL.
 * Every stage solves with its own factors (no lagged factors, no GMRES base solves);
 * the fallbacks of shoot_eval apply to the whole segmented march.  Synchronises.
 * Errors: WW_ENOSETUP, WW_EINVAL (a segment out of range, fractions not summing to 1,
 * the mesh rule, segs[0].N differing from shoot_setup's N), WW_EPIVOT, WW_ENONFINITE,
 * WW_EDOMAIN, WW_EREFINE (WW_STRICT), WW_EHIP.
 */
int shoot_eval_segments(ww_ctx *ctx, const double *params, double T, int nseg, const ww_segment *segs,
                        double *r, double *J, double *drdT, double *f);

/*
 * shoot_eval_segments_sdc: shoot_eval_segments with every segment's nsteps_l steps taken
 * by SDC15 (as shoot_eval_sdc) instead of DOP853: the combination the paper uses for its
 * sharp-crested waves (Sec. 2.2).  Arguments, regridding, outputs and errors as
 * shoot_eval_segments; step counts as for shoot_eval_sdc (the explicit scheme's dt must
 * resolve the largest frequency each segment's filter passes).  Synchronises.
 */
int shoot_eval_segments_sdc(ww_ctx *ctx, const double *params, double T, int nseg, const ww_segment *segs,
                            double *r, double *J, double *drdT, double *f);

/*
 * shoot_eval_batch: shoot_eval for n_inst independent instances (continuation
 * instances of uneven N, depth, tension, M and step count), each with its own context
 * (distinct contexts; give them distinct streams for the instances to overlap).  Each
 * context replays a captured step graph on its stream and the steps of all instances
 * are issued interleaved.  With more than one instance the step graphs keep each
 * instance on its one stream (the column chain follows the base chain), which lets the
 * GPU overlap the instances; a single instance is marched as by shoot_eval.  Per-instance arrays: params[i] (device),
 * T[i], nsteps[i] (host), r[i] (device), J[i] (device or NULL; J may be NULL),
 * drdT[i] (device or NULL; drdT may be NULL), f[i] (host; f may be NULL).
 * Results are identical to n_inst separate shoot_eval calls: an instance whose march
 * needs a fallback is redone alone as shoot_eval would.  Synchronises every context's
 * stream; returns the first instance error.
 */
int shoot_eval_batch(int n_inst, ww_ctx *const *ctx, const double *const *params, const double *T,
                     const int *nsteps, double *const *r, double *const *J, double *const *drdT,
                     double *f);

/*
 * shoot_adjoint (Sec. 3.2, App. B; discrete form): gradient of f = r.r/2 with respect
 * to the parameters, grad = J^T r, by the exact transpose of the discretised
 * variational march (reverse Runge-Kutta stages, transposed LU solves, transposed
 * Gm, -d/dx, -H), with the base state recomputed from checkpoints taken every
 * `ckpt_every` steps.  The factors are FP64 also in a WW_MIXED context.  Device
 * workspace for the checkpoints and for the factors of one segment (ckpt_every x stages
 * x 3 Np^2 doubles) is allocated on the first call and kept until ww_destroy.
 * grad: device M.  dfdT (host or NULL): df/dT = r . drdT.  f (host or NULL).
 * Synchronises.  A pivot below the guard redoes the call with partial pivoting.
 * Errors: WW_ENOSETUP, WW_EINVAL, WW_EPIVOT, WW_ENONFINITE, WW_EHIP.
 */
int shoot_adjoint(ww_ctx *ctx, const double *params, double T, int nsteps, int ckpt_every,
                  double *grad, double *dfdT, double *f);

/*
 * Measurement hooks (not part of the method): ww_profile(ctx, 1) adds timestamp nodes
 * (a one-thread kernel reading the GPU's constant-rate wall clock) around three phases
 * of every stage of the step graph -- 0: the block LU of A (a launch sequence, which in
 * a lagged-factor march factors a group of stages, with the block-triangular inverses
 * and the explicit inverse), 1: the whole base chain (spectral prep, assembly, base
 * solve, base DtN, base right-hand side), 2: the column chain (the M variational
 * columns) -- and clears the accumulated sums (stream-ordered); phase 3 is the host
 * time spent enqueueing one step (graph launches and event operations).  With 2 added
 * to `enable` (enable = 3), every block-LU step kernel (k_blu_step) that a march step
 * launches directly (not from a graph) also carries a pair of HIP events attached to its
 * dispatch on its stream (hipExtLaunchKernel), which take the kernel's own start and end
 * times; phase 4 reads their mean elapsed time (the kernel's average launch duration,
 * over at most the first 16384 launches of the interval).
 * ww_profile_read returns in *avg_ms the mean duration of `phase` over every interval
 * since the last ww_profile(ctx, 1) (per step for phase 3, per launch for phase 4), and
 * in *count the number of intervals (synchronises the stream).  Errors: WW_EINVAL (profiling off, nothing
 * replayed yet), WW_EHIP.
 */
int ww_profile(ww_ctx *ctx, int enable);
int ww_profile_read(ww_ctx *ctx, int phase, double *avg_ms, int *count);

/*
 * ww_fallbacks: in *bits, the fallbacks behind the results of the last successful
 * dtn_setup, dtn_solve_multi, shoot_eval or shoot_adjoint on this context (for
 * shoot_eval_batch: of that context's instance): WW_FB_PIVOTED, WW_FB_FP64, or 0 when
 * the results come from the context's own path.  Host only.  Errors: WW_EINVAL.
 */
int ww_fallbacks(ww_ctx *ctx, unsigned *bits);

/*
 * ww_thin_svd (App. C: J = U S V^T): thin singular value decomposition of the tall
 * matrix A (device, N x n column-major, ld N; 1 <= n <= N <= n_max, n <= r_max) by
 * one-sided Jacobi rotations on the GPU (sweeps until every column pair is orthogonal
 * to 1e-15 relative).  sigma (host, n): singular values in descending order.  V (host,
 * n x n column-major, or NULL): right singular vectors.  U (device, N x n, or NULL):
 * left singular vectors (zero column for a zero singular value).  A is not modified.
 * Synchronises.  Errors: WW_EINVAL, WW_ENONFINITE (non-finite entry), WW_ENOCONV,
 * WW_EHIP.
 */
int ww_thin_svd(ww_ctx *ctx, const double *A, int N, int n, double *sigma, double *V, double *U);

/*
 * Levenberg-Marquardt trust-region driver with delayed Jacobian updates (Sec. 3.3,
 * App. C) on the shooting problem of shoot_setup: it minimises f(c) = r.r/2 over
 * c = (T, params[0..M-1]), with the residual r and the Jacobian [dr/dT | dr/dparams]
 * from shoot_eval (nsteps steps, dt = T / (4 nsteps)).  Each trust-region subproblem is
 * solved through the thin SVD of J (eq. (trust:tilde)) by Newton's method on
 * tau(lambda) = 1/||p~|| - 1/Delta; J is re-used over accepted steps and re-computed
 * by the rules of App. C (1-4) with the parameters of ww_lm_opts.  Singular values below
 * (M + 1) eps sigma_max count as zero.
 * c (host, M + 1): T, then the parameters; the starting point on entry, the result on
 * return.  opts: NULL for the defaults (ww_lm_default_opts).  rep (or NULL): the final
 * f and radius, evaluation counts, the reason of termination (WW_LM_*), and optionally
 * the history of tried steps: rows of (c_new[M + 1], f(c_new), accepted) in
 * history (host, hist_cap rows of M + 3 doubles; n_hist counts every tried step).
 * Synchronises.  Errors: those of shoot_eval and ww_thin_svd, WW_ENOSETUP, WW_EINVAL.
 */
typedef struct ww_lm_opts {
  double f_tol;       /* roundoff regime when f < f_tol (App. C: 1e-26) */
  double g_tol;       /* ... or Delta < g_tol, or on a fresh J ||g|| < g_tol (1e-13) */
  double df_tol;      /* ... or on a fresh J |df|/f < df_tol; J re-computation (1e-5) */
  double delta0;      /* initial trust-region radius (0.1) */
  int max_steps_J;    /* accepted steps per Jacobian (10) */
  int max_evals;      /* cap on residual + Jacobian evaluations (200) */
} ww_lm_opts;

typedef struct ww_lm_report {
  double f, delta;
  int evals_r, evals_J, reason, n_hist;
  double *history;    /* host, or NULL */
  int hist_cap;
} ww_lm_report;

#define WW_LM_F_ZERO 1
#define WW_LM_C_UNCHANGED 2
#define WW_LM_ROUNDOFF_REJECTED 3
#define WW_LM_ROUNDOFF_MAX_STEPS_J 4
#define WW_LM_MAX_EVALS 5

int ww_lm_default_opts(ww_lm_opts *opts);
int ww_levmar(ww_ctx *ctx, double *c, int nsteps, const ww_lm_opts *opts, ww_lm_report *rep);

/*
 * BFGS minimiser with the adjoint gradient (the ACM of Sec. 3.2) on the shooting
 * problem of shoot_setup: it minimises f(c) = r.r/2 over c = (T, params[0..M-1]) with
 * f and grad f = (df/dT, grad_params f) from shoot_adjoint (checkpoints every
 * ckpt_every steps).  The paper names BFGS with line searches; its parameters here:
 * inverse-Hessian update H <- (I - rho s y^T) H (I - rho y s^T) + rho s s^T (skipped when
 * y.s <= 0), H_0 = I scaled by s.y / y.y at the first update; strong Wolfe line search
 * (c1 = 1e-4, c2 = 0.9) with first trial step 1 (capped at a length delta0 on the first
 * iteration), bracketing by doubling (at most 20) and zoom by bisection (at most 30); a
 * search without the conditions takes the best point met if it lowers f, else stops.
 * c (host, M + 1): start on entry, result on return.  opts: NULL for the defaults.  rep
 * (or NULL): final f and ||g||, iterations, evaluations (f and gradient), reason
 * (WW_BFGS_*), and optionally rows of (c[M + 1], f) after every iteration in history
 * (host, hist_cap rows of M + 2 doubles).  Synchronises.  Errors: those of
 * shoot_adjoint, WW_ENOSETUP, WW_EINVAL.
 */
typedef struct ww_bfgs_opts {
  double f_tol;     /* stop when f < f_tol (1e-26) */
  double g_tol;     /* ... or ||grad f|| < g_tol (1e-13) */
  double delta0;    /* length cap of the first step (0.1) */
  int max_iter;     /* (200) */
  int ckpt_every;   /* adjoint checkpoints (16) */
} ww_bfgs_opts;

typedef struct ww_bfgs_report {
  double f, gnorm;
  int iters, evals, reason, n_hist;
  double *history;  /* host, or NULL */
  int hist_cap;
} ww_bfgs_report;

#define WW_BFGS_F_TOL 1
#define WW_BFGS_G_TOL 2
#define WW_BFGS_C_UNCHANGED 3
#define WW_BFGS_LINE_SEARCH 4
#define WW_BFGS_MAX_ITER 5

int ww_bfgs_default_opts(ww_bfgs_opts *opts);
int ww_bfgs(ww_ctx *ctx, double *c, int nsteps, const ww_bfgs_opts *opts, ww_bfgs_report *rep);

/*
 * ww_next_fallback (host only, no context): the decision a march takes from its status
 * bits -- 1 pivot below the guard (unpivoted LU), 8 pivot below the guard (pivoted LU),
 * 2 non-finite state, 4 failed refinement test (mixed form), 16 surface through the
 * bottom, 32 failed test of a lagged-factor solve, 64 failed test of a GMRES solve --
 * for a context with `flags` (WW_STRICT matters) whose current results came from the
 * fallbacks `fb` (WW_FB_* bits): the WW_FB_* bits to add and redo the march with, or 0
 * (report the status as an error, or succeed).  A small pivot is redone with pivoted
 * factors first (every stage then solves with its own factors).  A failed lagged or
 * GMRES solve is redone on each stage's own factors before a bed crossing is reported
 * (the crossing may come from the unconverged solves); a crossing on those factors
 * ends the call with WW_EDOMAIN.  Exposed for tests of the host logic.
 */
unsigned ww_next_fallback(unsigned flags, unsigned fb, int status);

/*
 * Launch and scheduling choices of a context (none changes what is computed, only how
 * the work is cut into launches and streams; the defaults are those of ww_create, or of
 * the WW_* environment knobs read there).  The project's autotuner
 * (paper_1210_5672_amd/autotune.py) times short marches over these choices and keeps
 * the fastest per (N, M, precision, GPU architecture) in a JSON cache.
 *   lag          lagged-factor march: the base solve of stage s uses the explicit
 *                inverse of stage s - lag (0: each stage's own factors), 0..11
 *   lu_group     consecutive stages factored by one launch sequence, 1..4 (<= lag)
 *   lu_streams   streams the LU groups rotate over, 1..6
 *   graph_parts  march parts replayed from HIP graphs, one bit each: 1 prep and
 *                assembly, 2 LU, 4 base chain, 8 column chain (the rest launched
 *                directly), 0..15
 *   minv_wgs     workgroup cap of the explicit-inverse launch, >= 1
 *   blu_strip    64-tiles per task of a block-LU step, 1..16
 *   dtn_rows     rows per workgroup of the base DtN launch, 4..32, a multiple of 4
 *   gemm_split   wave groups splitting the inner dimension of a column product, 2 or 4
 *   gemm_rows    rows of a column product's output tile, 16 or 32 (16: twice the
 *                workgroups for the same columns)
 *   lag_fp32     FP64 form, lagged-factor march: 1 makes the lagged base solve (its
 *                first solve and the corrections of its refinement sweeps) read an FP32
 *                copy of the lagged inverse, written by the same launch as the FP64 one;
 *                the residuals stay FP64 and the solve still ends with the 2^-43 test, so
 *                only the contraction per sweep changes (half the bytes per product)
 *   asm_cw       columns per assembly workgroup, 16 or 32
 *   lag_sweeps   refinement sweeps of a lagged-factor base solve, 1..8 (default 2, or
 *                WW_NREF_LAG); each sweep multiplies the error by about
 *                ||A_old^-1 A - I||, so marches whose matrix moves faster per step need
 *                more of them to pass the 2^-43 test (else they fall back)
 * ww_set_tuning validates every field and applies them together (captured graphs are
 * re-captured at the next march); ww_get_tuning reads the current choices.  Host only.
 * Errors: WW_EINVAL (null argument, a field out of range).
 */
typedef struct ww_tuning {
  int lag, lu_group, lu_streams, graph_parts, minv_wgs, blu_strip, dtn_rows, gemm_split, asm_cw, gemm_rows,
      lag_fp32, lag_sweeps;
} ww_tuning;
int ww_get_tuning(ww_ctx *ctx, ww_tuning *t);
int ww_set_tuning(ww_ctx *ctx, const ww_tuning *t);

/* thread-local message of the last failure on this thread ("" if none) */
const char *ww_last_error(void);

/* library version string */
const char *ww_version(void);

#ifdef __cplusplus
}
#endif

#endif /* WW_H */
