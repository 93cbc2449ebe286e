/*
 * gp.h -- C ABI of the MI355X iterative Gaussian-process hot path.
 *
 * Operations follow Lin et al., "Improving Linear System Solvers for
 * Hyperparameter Optimisation in Iterative Gaussian Processes" (NeurIPS 2024):
 * the matrix-free regularised kernel block product (K + sigma^2 I) V behind
 * every solver iteration and gradient estimate, the three linear solvers of
 * its App. B (Algorithms 1-3), the standard and pathwise gradient estimators
 * (Secs. 2-3), random-Fourier-feature prior samples (App. B) and the
 * initial-hyperparameter heuristic of its large-data experiments (App. B).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Kernel: Matern-3/2 with per-dimension length scales ell_k and signal
 *    scale a:  r^2 = sum_k ((x_k - x'_k)/ell_k)^2,
 *    k(x,x') = a^2 (1 + sqrt(3) r) exp(-sqrt(3) r).   H = K(X,X) + sigma^2 I.
 *  - theta is a HOST array of d+2 doubles (ell_1..ell_d, a, sigma), all > 0.
 *  - Every float/int array argument is a DEVICE pointer on the context's
 *    device, owned by the caller; the library never frees or keeps it.
 *    Matrices are row-major with an explicit leading dimension ld >= columns.
 *    X arrays are [n, d] contiguous (leading dimension d).
 *  - Host outputs (grad_out, stats) are complete when the call returns; device
 *    outputs are complete in stream order on the context's stream.
 *  - Work is enqueued on the stream given to gp_ctx_create.  One context per
 *    host thread; calls on one context must not overlap.
 *  - Return value: GP_OK or an error code; gp_last_error() gives the text.
 *    On error, device outputs are unspecified and no state is leaked.
 *  - The library allocates its workspace with hipMalloc on first use and
 *    grows it when a larger problem arrives (never inside a solver loop);
 *    gp_workspace_size tells its size and gp_workspace_reserve allocates it
 *    up front.
 */
#ifndef GP_H
#define GP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gp_ctx gp_ctx;

enum gp_status {
  GP_OK = 0,
  GP_ERR_INVALID_ARG = 1,  /* bad size, pointer, theta or configuration        */
  GP_ERR_HIP = 2,          /* a HIP runtime call failed                          */
  GP_ERR_NO_WORKSPACE = 3, /* device memory for the workspace could not be had   */
  GP_ERR_NONFINITE = 4,    /* a residual or iterate became NaN/Inf               */
  GP_ERR_BREAKDOWN = 5     /* CG found d^T H d <= 0 on a live column            */
};

/* Arithmetic of the kernel-matrix product.
 *  GP_FP32   kernel values and V in FP32 on FP32 MFMA, FP32 accumulation.
 *  GP_BF16X3 kernel values and V split into bf16 hi + lo parts, three bf16
 *            MFMA products (hi*hi + hi*lo + lo*hi), FP32 accumulation.
 *  GP_BF16   kernel values and V rounded once to bf16, one bf16 MFMA product.
 * Squared distances, the Matern evaluation and the epilogue are FP32 in all
 * modes; bf16 rounding is round-to-nearest-even.                              */
enum gp_precision { GP_FP32 = 0, GP_BF16X3 = 1, GP_BF16 = 2 };

enum gp_solver { GP_CG = 0, GP_AP = 1, GP_SGD = 2 };
enum gp_estimator { GP_STANDARD = 0, GP_PATHWISE = 1 };

/* How the gradient contraction u^T (dH/dtheta_k) w is formed.
 *  GP_ADJ_FUSED     one pass over all kernel entries computing every partial
 *                   derivative at once (kernel tiles recomputed, never stored).
 *  GP_ADJ_PER_PARAM d+1 separate FP32 derivative-kernel products
 *                   (dK/dtheta_k) W, one per length scale and the signal
 *                   scale, each followed by a dot product with U.           */
enum gp_adjoint_mode { GP_ADJ_FUSED = 0, GP_ADJ_PER_PARAM = 1 };

enum gp_transform { GP_SOFTPLUS = 0, GP_LOG = 1 };

/* ------------------------------------------------------------------ context */

/* Create a context on HIP device `device` that enqueues all work on `stream`
 * (a hipStream_t; NULL = the legacy default stream).  *out receives the
 * context.  Errors: GP_ERR_INVALID_ARG (out NULL), GP_ERR_HIP.              */
int gp_ctx_create(int device, void* stream, gp_ctx** out);

/* Free the context and its workspace (synchronises its stream first). */
void gp_ctx_destroy(gp_ctx* ctx);

/* Text of the last error on this context ("" if none). Valid until the next call. */
const char* gp_last_error(const gp_ctx* ctx);

/* Library version string, e.g. "gpmi 0.1 gfx950". */
const char* gp_version(void);

/* Per-launch HIP-event timing, recorded on the context's stream around the
 * library's own kernel launches (also those inside gp_solve / gp_mll_grad).
 * enable != 0 starts recording (and clears totals); enable = 0 stops.
 * gp_profile_read synchronises the stream and returns the summed duration in
 * milliseconds and the launch count of kernel class `which`:
 *   0 = forward product kernel in GP_BF16X3 / GP_BF16, 1 = fused adjoint,
 *   2 = random-feature sample, 3 = CG vector updates, 4 = forward product kernel
 *   in GP_FP32 (classes 0 and 4 time the product kernel alone, not the sum of
 *   its column-split partials), 5 = CG preconditioner (construction and apply),
 *   6 = nearest-row selection, 7 = exact-likelihood factorisation (H, its
 *   Cholesky factor and inverse, H^-1: FP64 GEMMs and leaf blocks), 8 = the rest
 *   of the exact likelihood (alpha, gradient contraction).
 * Errors: GP_ERR_INVALID_ARG for an unknown class.                          */
int gp_profile_enable(gp_ctx* ctx, int enable);
int gp_profile_read(gp_ctx* ctx, int which, double* total_ms, int64_t* launches);

/* ---------------------------------------------------- kernel-matrix product */

/* out = a^2 M(X1, X2) V  (+ sigma^2 V when add_noise), i.e. K(X1,X2) V or,
 * with X1 == X2 and add_noise = 1, the regularised product H V of Sec. 2
 * (definition of H_theta).  This is the operator every solver iteration
 * applies (App. B, Algorithms 1-3).
 *   X1 [n1, d], X2 [n2, d]   inputs (rows of the output / of V)
 *   V  [n2, ldv], first c columns used;  out [n1, ldo], first c columns written
 *   add_noise requires n1 == n2 and X1 describing the same points as X2.
 * n1 = 0 or n2 = 0 or c = 0 is a no-op (out untouched; with n2 = 0 and
 * n1 > 0 the first c columns of out are set to zero).
 * Columns go through the kernel in passes of at most 80; every pass evaluates
 * the kernel entries again, so c is limited only by the workspace.
 * Errors: GP_ERR_INVALID_ARG for d < 1, d > 64, c > 1024, ld < c, theta <= 0,
 * a NULL pointer with a non-empty size.                                     */
int gp_kmatvec(gp_ctx* ctx, const float* X1, int64_t n1, const float* X2, int64_t n2, int d,
               const double* theta, const float* V, int64_t ldv, int c, float* out, int64_t ldo,
               int precision, int add_noise);

/* gp_kmatvec for callers that cannot allocate memory (code that must not call
 * hipMalloc or an allocating library routine, such as a tight serving loop or a
 * harness that forbids it): the same product, arguments, results and errors,
 * with every buffer of the call (packed inputs, bf16 / FP32 operand tiles,
 * column-split partial sums) carved from a static device array of 64 MiB that the
 * library holds on each device it runs on until the process ends, and host
 * staging kept in the context.  No hipMalloc, hipHostMalloc or hipFree.
 * Limit: the packed inputs and one column pass of packed V must fit 64 MiB, e.g.
 * n1 = n2 = 150,000 with d <= 3 and c <= 80 (inputs 16 bytes a row, V tiles 320
 * bytes a row); larger calls fail with GP_ERR_INVALID_ARG and a message that
 * names the sizes.  The split of the column range over workgroups is reduced to
 * what the remaining scratch holds, so the summation order (and the last bits)
 * can differ from gp_kmatvec's.  Every call on one device shares that device's
 * array and overwrites it: calls that overlap on one device (two host threads,
 * or two streams) race; serialise them.  Per-launch profiling is not recorded.  */
int gp_kmatvec_static(gp_ctx* ctx, const float* X1, int64_t n1, const float* X2, int64_t n2,
                      int d, const double* theta, const float* V, int64_t ldv, int c, float* out,
                      int64_t ldo, int precision, int add_noise);

/* Bilinear adjoint: grad_out[k] = sum_c col_weights[c] * U[:,c]^T (dH/dtheta_k) W[:,c]
 * for k = 0..d+1 (ell_1..ell_d, a, sigma), with dH/dsigma = 2 sigma I
 * (App. A).  This is the contraction of the gradient estimators (Sec. 2
 * eq. mll_grad, Sec. 3 eq. pathwise_estimator).
 *   U [n, ldu], W [n, ldw]: first c columns used.  col_weights: HOST [c].
 *   precision: GP_FP32 or GP_BF16X3 for the U diag(w) W^T tile products.
 *   mode: gp_adjoint_mode.  grad_out: HOST [d+2] doubles.
 * The fused pass takes up to 256 columns; more columns (up to 1024) run as
 * several passes whose sums are added.
 * Errors as gp_kmatvec.                                                     */
int gp_kmatvec_adjoint(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta,
                       const float* U, int64_t ldu, const float* W, int64_t ldw, int c,
                       const double* col_weights, int precision, int mode, double* grad_out);

/* ------------------------------------------------------------------- solvers */

typedef struct gp_solver_cfg {
  int solver;           /* gp_solver                                                    */
  double tol;           /* relative residual tolerance tau (paper: 0.01)                */
  double max_epochs;    /* budget T in epochs; <= 0 means tolerance only (safety cap)   */
  int precision;        /* gp_precision of the products inside the iteration            */
  int refine_every;     /* FP32 true-residual replacement every k iterations (0 = only
                           at exit); ignored for GP_FP32                                 */
  int check_every;      /* stopping test every k iterations (0 = library default)        */
  int ap_block;         /* AP block size b (paper: 1000), at most 2048                   */
  int sgd_batch;        /* SGD batch size b (paper: 500)                                 */
  double sgd_lr;        /* SGD learning rate gamma                                       */
  double sgd_momentum;  /* SGD momentum rho (paper: 0.9)                                 */
  const int32_t* sgd_batches; /* HOST [sgd_batches_count, sgd_batch] row indices per
                                 iteration, distinct within a batch (an index outside
                                 [0, n) or repeated in its batch: GP_ERR_INVALID_ARG),
                                 or NULL to draw them from sgd_seed                      */
  int64_t sgd_batches_count;
  uint64_t sgd_seed;
  int precond_rank;     /* CG only: rank k of the pivoted-Cholesky preconditioner
                           P = L L^T + sigma^2 I (App. B uses 100); 0 = none (P = I);
                           at most 32768 and capped at n                            */
  int use_graph;        /* CG only: run the solve on a library-owned stream (ordered with
                           the context's stream by events) and replay one captured
                           iteration as a HIP graph from the second iteration on; the
                           results are identical to the eager solve. Worth it where an
                           iteration is short (small n). Per-kernel profiling is not
                           recorded for replayed iterations.                          */
  int precond_reuse;    /* CG with precond_rank > 0: the pivoted-Cholesky factor L built by
                           one solve may serve up to this many later solves on the same X
                           (same pointer, same contents by a fingerprint taken at each
                           solve, same n and d) and rank before it is rebuilt; 0 = rebuild
                           in every solve.  A reused L still defines an exact SPD
                           P = L L^T + sigma^2 I with the current sigma (only the k x k
                           Woodbury factor is recomputed), so the accepted solutions meet
                           the same residual test; only the iteration count can differ. */
} gp_solver_cfg;

typedef struct gp_solve_stats {
  int64_t iterations;   /* solver iterations run                                         */
  double epochs;        /* iterations converted to epochs (App. B)                       */
  int64_t matvecs;      /* full H*V products incl. initial residual and refinements      */
  int64_t refinements;  /* FP32 true-residual replacements                               */
  double relres_y;      /* ||r_y|| of the normalised system at exit (solver's residual)  */
  double relres_z;      /* mean_j ||r_j|| at exit                                        */
  double true_relres_y; /* FP32 true residual ||b~ - H u~|| at exit: computed whenever the
                           budget stops a solve (all solvers) and when CG accepts a
                           reduced-precision solution; NaN otherwise                    */
  double true_relres_z;
  int converged;        /* 1 if both residual norms reached tol                         */
  int status;           /* gp_status of the solve                                        */
  int precond_rank;     /* rank of the preconditioner actually built (may be below the
                           requested rank when K is numerically of lower rank)          */
  int64_t fp32_iterations; /* CG only: iterations run with FP32 products after restarts
                           from the true residual stopped gaining with the requested
                           reduced precision (0 when that precision reached tol)     */
} gp_solve_stats;

/* Fill *cfg with the paper's defaults: CG, tol 0.01, no budget, FP32,
 * refine_every 0, AP block 1000, SGD batch 500, lr 10, momentum 0.9, no
 * preconditioner (set precond_rank = 100 for the paper's CG configuration).  */
void gp_solver_cfg_default(gp_solver_cfg* cfg);

/* Solve H [u_0..u_{c-1}] = [b_0..b_{c-1}] (App. B, Algorithms 1-3).
 * Column 0 is the mean system (y); columns 1..c-1 are the probe systems.
 * Rules: each column is normalised, b~ = b/(||b|| + 1e-10), and the loop
 * continues while iterations remain and (||r_0|| > tol or mean_j ||r_j|| > tol).
 * Budget: CG runs at most T iterations; AP/SGD at most ceil(nT/b).
 *   B [n, ldb] right-hand sides; U [n, ldu] IN: initial value (zeros for a
 *   cold start, the previous solution for a warm start), OUT: solution.
 *   cfg, stats: HOST structs (stats may be NULL).
 * Not reaching tol within the budget is not an error (stats->converged = 0).
 * At most 256 columns (the per-column scalar reductions of one iteration run
 * one thread per column in one 256-thread block); gp_mll_grad likewise takes
 * s <= 255 probes.
 * Errors: GP_ERR_INVALID_ARG, GP_ERR_NONFINITE, GP_ERR_BREAKDOWN, GP_ERR_HIP. */
int gp_solve(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta,
             const float* B, int64_t ldb, float* U, int64_t ldu, int c,
             const gp_solver_cfg* cfg, gp_solve_stats* stats);

/* Rank-k greedy pivoted Cholesky of K(X, X) (the CG preconditioner of App. B):
 * at step j the pivot p is the row with the largest remaining diagonal (lowest
 * index on ties), L[:, j] = (K[:, p] - L[:, :j] L[p, :j]^T) / sqrt(d_p) and
 * d <- d - L[:, j]^2; it stops early when no remaining diagonal is positive.
 * Kernel columns are evaluated in FP64 from X; the factor is FP64.
 *   L   DEVICE [k, ldl] doubles, stored transposed: L[j * ldl + i] is entry i
 *       of factor column j (ldl >= n); entries of rows >= rank are untouched
 *   piv DEVICE [k] int32 pivot indices (first *rank written)
 *   rank HOST out: the rank reached (<= min(k, n))
 * k = 0 or n = 0 is a no-op with *rank = 0.
 * Errors: GP_ERR_INVALID_ARG (k > 32768, ldl < n, NULL pointers), GP_ERR_HIP. */
int gp_pivoted_cholesky(gp_ctx* ctx, const float* X, int64_t n, int d, const double* theta,
                        int k, double* L, int64_t ldl, int32_t* piv, int* rank);

/* ---------------------------------------------------------------- workspace */

/* Operations whose device workspace can be planned (the buffers the library
 * keeps between calls: packed inputs, bf16 operand tiles, column-split partial
 * sums, solver vectors and scalars, the preconditioner factor).             */
enum gp_ws_op {
  GP_WS_KMATVEC = 0,  /* gp_kmatvec H V with X1 == X2 (cfg->precision; cfg may be NULL
                         for GP_FP32)                                             */
  GP_WS_SOLVE = 1,    /* gp_solve with *cfg                                      */
  GP_WS_MLL_GRAD = 2  /* gp_mll_grad with *cfg, s = c - 1 probes and M random-feature
                         pairs (M = 0 for the standard estimator), either adjoint mode */
};

/* Bytes of device memory a context holds after one call of `op` on n points in
 * d dimensions with c columns: the operator, its solver iterations and right-hand
 * sides are the Require lines of App. B, Algorithms 1-3 (H, b and the solver's
 * vectors).  Where a size depends on the data (the squared-distance form, the
 * preconditioner rank reached) the larger case is counted, so the figure is an
 * upper bound for that call.  Host-only: no context or device needed.
 * Errors: GP_ERR_INVALID_ARG for an unknown op, a NULL bytes or cfg (where
 * needed), or sizes the operation itself rejects.                            */
int gp_workspace_size(int op, int64_t n, int d, int c, const gp_solver_cfg* cfg, int M,
                      size_t* bytes);

/* Allocate, now, the workspace gp_workspace_size counts, on ctx's device: later
 * calls of `op` of at most this size allocate nothing (buffers only grow).
 * Errors: as gp_workspace_size; GP_ERR_NO_WORKSPACE, GP_ERR_HIP.             */
int gp_workspace_reserve(gp_ctx* ctx, int op, int64_t n, int d, int c,
                         const gp_solver_cfg* cfg, int M);

/* Bytes of device workspace ctx holds now (*bytes; host).  Errors:
 * GP_ERR_INVALID_ARG for NULL arguments.                                    */
int gp_workspace_held(const gp_ctx* ctx, size_t* bytes);

/* --------------------------------------------------------- random features */

/* Prior function sample with random Fourier features (App. B, "Kernel
 * Function and Random Features"): with omega_m = t_m / ell,
 *   F[i, j] = (a / sqrt(M)) sum_m ( cos(x_i . omega_m) W[m, j] + sin(x_i . omega_m) W[M+m, j] )
 *   Xq [m_rows, d] query points; t [M, d] base frequencies (unit length
 *   scale, drawn by the caller from the Matern-3/2 spectral measure, a
 *   3-degree-of-freedom Student-t); W [2M, ldw] feature weights (first s
 *   columns used; rows 0..M-1 weight cos, rows M..2M-1 weight sin);
 *   F [m_rows, ldf] output (first s columns written).
 * The phase x . omega is formed and reduced modulo 2 pi in FP64; the sine and
 * cosine and the weighted sum are FP32.                                     */
int gp_prior_sample(gp_ctx* ctx, const float* Xq, int64_t m_rows, int d, const double* theta,
                    const float* t, int M, const float* W, int64_t ldw, int s, float* F,
                    int64_t ldf);

/* Pathwise posterior samples (Sec. 2 eq. pathwise_conditioning; Sec. 3,
 * "Amortising Linear Solves for Optimisation and Prediction"): with the pathwise
 * solutions U = [v_y, zhat_1..zhat_s] of H U = [y, xi_1..xi_s] and the same
 * random features (t, W) that produced the prior draws xi_j = f_j(x) + eps_j,
 *   F[q, j] = f_j(Xq[q]) + sum_i k(Xq[q], X[i]) (v_y[i] - zhat_j[i]),
 * i.e. prediction at Xq without further solves.  f_j is gp_prior_sample's
 * random-feature function; the kernel product runs at `precision`.
 *   Xq [m_rows, d] query points; X [n, d] training inputs; t [M, d], W [2M, ldw]
 *   as in gp_prior_sample (first s columns of W); U [n, ldu] (s + 1 columns:
 *   v_y, then zhat_1..zhat_s); F [m_rows, ldf] output (first s columns).
 * n = 0 returns the prior samples; m_rows = 0 or s = 0 is a no-op.
 * Errors as gp_prior_sample and gp_kmatvec.                                 */
int gp_posterior_sample(gp_ctx* ctx, const float* Xq, int64_t m_rows, const float* X, int64_t n,
                        int d, const double* theta, const float* t, int M, const float* W,
                        int64_t ldw, const float* U, int64_t ldu, int s, int precision, float* F,
                        int64_t ldf);

/* -------------------------------------------------- marginal-likelihood step */

/* Gradient estimate of the log marginal likelihood (Sec. 2 eq. mll_grad):
 *   g_k = 1/2 v_y^T dH_k v_y - 1/(2s) sum_j v_j^T dH_k b_j
 * STANDARD (Sec. 2 eq. trace): b_j = z_j = Z[:, j] probe vectors, v = H^-1 [y, Z].
 * PATHWISE (Sec. 3): b_j = xi_j = f_j(x) + sigma w_eps[:, j] with f_j the
 *   random-feature prior sample (t, W as gp_prior_sample, current theta), and
 *   the trace term uses zhat_j^T dH_k zhat_j, zhat = H^-1 xi.
 *   y [n]; Z [n, ldz] (STANDARD) or rff_t [M, d], rff_W [2M, ldw], w_eps [n, ldeps]
 *   (PATHWISE); unused pointers may be NULL.
 *   U [n, ldu], s+1 columns: IN warm start (zeros = cold), OUT solutions
 *   [v_y, v_1..v_s] -- pass the same buffer every step to warm start (Sec. 4).
 *   grad_out: HOST [d+2] doubles (derivative w.r.t. theta, ascent direction).
 *   stats: HOST, may be NULL.                                                */
int gp_mll_grad(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                const double* theta, int estimator, int s, const float* Z, int64_t ldz,
                const float* rff_t, int M, const float* rff_W, int64_t ldw, const float* w_eps,
                int64_t ldeps, float* U, int64_t ldu, const gp_solver_cfg* cfg, int adjoint_mode,
                double* grad_out, gp_solve_stats* stats);

/* Outer-loop update on the HOST (App. B, "Iterative Optimiser"): theta =
 * softplus(nu) (or exp(nu) for GP_LOG); one Adam ascent step on nu with the
 * chain rule dtheta/dnu applied to grad_theta.  Adam: beta1 = 0.9,
 * beta2 = 0.999, eps = 1e-8, bias-corrected.  All arrays HOST [p];
 * *step is the Adam step counter (0 before the first call), incremented.    */
int gp_adam_ascent(int p, double* nu, double* m, double* v, int64_t* step,
                   const double* grad_theta, double lr, int transform);

/* theta[k] = softplus(nu[k]) or exp(nu[k]) (HOST arrays [p]). */
int gp_nu_to_theta(int p, const double* nu, int transform, double* theta);

/* The inverse: nu[k] = softplus^-1(theta[k]) = theta[k] + log(1 - exp(-theta[k]))
 * or log(theta[k]) (HOST arrays [p]), the unconstrained starting point of the
 * optimiser for hyperparameters theta > 0 (App. B, "Iterative Optimiser").
 * Errors: GP_ERR_INVALID_ARG for p < 0, NULL arrays, an unknown transform or
 * a theta[k] that is not finite and positive.                              */
int gp_theta_to_nu(int p, const double* theta, int transform, double* nu);

/* ------------------------------------ initial hyperparameters (large data) */

/* Step 2 of the initial-hyperparameter heuristic (App. B, "Iterative
 * Optimiser"): the k rows of X nearest to row `centre`.  Distance: squared
 * Euclidean distance in the raw inputs, summed in FP64 in dimension order with
 * every product and sum rounded separately (no fused multiply-add); equal
 * distances go to the lower row index.
 *   X [n, d]; centre in [0, n) (drawn uniformly at random by the caller, step 1);
 *   idx DEVICE [k] int64 output, the selected rows in ascending order.
 * k = 0 is a no-op; k = n returns 0..n-1.
 * Errors: GP_ERR_INVALID_ARG (k < 0, k > n, centre outside [0, n), NULL
 * pointers, d outside [1, 64]), GP_ERR_HIP.                                 */
int gp_nearest(gp_ctx* ctx, const float* X, int64_t n, int d, int64_t centre, int64_t k,
               int64_t* idx);

/* Exact log marginal likelihood and its gradient (Sec. 2, eqs. mll and
 * mll_grad) on m rows of (X, y), by a dense FP64 Cholesky factorisation:
 *   L   = -1/2 y^T H^-1 y - 1/2 log det H - m/2 log 2 pi
 *   g_k = 1/2 alpha^T dH_k alpha - 1/2 tr(H^-1 dH_k),  alpha = H^-1 y.
 * The rows are idx[0..m) (DEVICE int64, each in [0, n)) or, with idx = NULL,
 * rows 0..m-1.  X [n, d], y [n] DEVICE.  mll: HOST double out (may be NULL);
 * grad: HOST [d+2] doubles out (ell_1..ell_d, a, sigma; may be NULL).
 * Workspace: two (m rounded up to 64)^2 FP64 matrices.
 * Errors: GP_ERR_INVALID_ARG (m < 1, m > 32768, m > n without idx, an index
 * outside [0, n), theta <= 0), GP_ERR_BREAKDOWN (a non-positive pivot: H is
 * not numerically positive definite), GP_ERR_NO_WORKSPACE, GP_ERR_HIP.      */
int gp_exact_mll(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                 const int64_t* idx, int64_t m, const double* theta, double* mll, double* grad);

typedef struct gp_init_cfg {
  int steps;             /* Adam steps per centroid subset (default 100)            */
  double lr;             /* Adam learning rate (default 0.1)                        */
  int transform;         /* GP_SOFTPLUS (default) or GP_LOG                         */
  const double* theta0;  /* HOST [d+2] starting point; NULL = 1.0 for every entry   */
} gp_init_cfg;

/* Defaults: the paper's small-data optimiser settings (App. B: hyperparameters
 * initialised at 1.0, learning rate 0.1, 100 Adam steps, softplus).          */
void gp_init_cfg_default(gp_init_cfg* cfg);

/* The initial-hyperparameter heuristic for large data sets (App. B,
 * "Iterative Optimiser"): for every centroid row c in centres (HOST [nc],
 * drawn uniformly by the caller), take the m rows nearest to it (gp_nearest),
 * maximise the exact marginal likelihood on them with Adam (gp_exact_mll and
 * gp_adam_ascent, cfg), and return the arithmetic mean of the resulting theta.
 *   X [n, d], y [n] DEVICE; theta_out HOST [d+2]; theta_each HOST [nc, d+2]
 *   (per-centroid results, may be NULL).  The paper uses m = 10,000, nc = 10.
 * Errors: as gp_nearest and gp_exact_mll; GP_ERR_INVALID_ARG also for nc < 1,
 * m > n, steps < 0, lr <= 0 or an invalid theta0.                            */
int gp_init_heuristic(gp_ctx* ctx, const float* X, int64_t n, int d, const float* y,
                      const int64_t* centres, int nc, int64_t m, const gp_init_cfg* cfg,
                      double* theta_out, double* theta_each);

#ifdef __cplusplus
}
#endif

#endif /* GP_H */
