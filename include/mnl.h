/*
 * mnl.h - C ABI of the GPU Newton-Raphson multinomial-logit fitter.
 *
 * Method: Hasan, Wang, Mahani, "Fast Estimation of Multinomial Logit Models:
 * R Package mnlogit" (arXiv:1404.3177).  One Newton-Raphson iteration is the
 * fused utility / probability / log-likelihood / gradient pass (Eqs. 2-5, 9),
 * the block-structured Hessian (Eq. 10), the Cholesky solve of the Newton
 * system (Eq. 6) and the step-halving line search (Sec. 3.1).
 *
 * Data kinds (this ABI's letters; the paper swaps Y and Z):
 *   X [N][p]     individual-specific data, alternative-specific coefficients
 *                beta_k (paper: X_i . beta_k).  An intercept is an X column
 *                of ones supplied by the caller, with alternative-specific
 *                coefficients like any other column of X (Sec. 3.1).
 *   Y [N][K][g]  alternative-varying data, generic coefficients alpha
 *                (paper: Z_ik . alpha).
 *   Z [N][K][a]  alternative-varying data, alternative-specific coefficients
 *                gamma_k (paper: Y_ik . gamma_k).
 * Alternative 0 is the base: beta_0 = 0 (Sec. 2.2 normalisation).  theta has
 * n_p = (K-1) p + K a + g entries in the Eq. 8 order
 *   theta = (beta_1 .. beta_{K-1}, gamma_0 .. gamma_{K-1}, alpha),
 * each chunk contiguous, features in column order within a chunk.
 *
 * Memory: every array argument is a DEVICE pointer owned by the caller
 * (row-major, float64 unless stated), except the host structs mnl_fit_opts
 * and mnl_fit_info.  The library keeps no pointer to caller memory after the
 * work it enqueued has completed.  It owns a per-context workspace in device
 * memory that grows on demand (hipMalloc) and is freed by mnl_destroy.
 * Work is enqueued on the given HIP stream (hipStream_t passed as void*,
 * NULL = the default stream); mnl_loglik_grad and mnl_hessian return without
 * synchronising, mnl_newton_step and mnl_fit synchronise the stream before
 * they return.  A context is used by one host thread at a time.
 *
 * Errors: functions return MNL_OK (0) or a negative MNL_ERR_* code; the
 * outputs are then unspecified.  mnl_strerror() names a code and
 * mnl_last_error() gives the context's last message.
 */
#ifndef MNL_H
#define MNL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MNL_VERSION_MAJOR 0
#define MNL_VERSION_MINOR 1

typedef struct mnl_ctx mnl_ctx;

/* Return codes. */
enum {
    MNL_OK = 0,
    MNL_ERR_ARG = -1,          /* bad dimension, NULL pointer, bad option,
                                  choice out of range (when validating)   */
    MNL_ERR_OOM = -2,          /* device allocation failed                */
    MNL_ERR_NOT_PD = -3,       /* -H not numerically positive definite    */
    MNL_ERR_NONFINITE = -4,    /* NaN/Inf in data or log-likelihood       */
    MNL_ERR_LS_FAIL = -5,      /* line search exhausted its halvings      */
    MNL_ERR_HIP = -6,          /* a HIP runtime call failed               */
    MNL_ERR_UNSUPPORTED = -7   /* shape beyond the kernels' limits        */
};

/* Stop reasons reported in mnl_fit_info.stop_reason.  The first three are
 * mnlogit's gtol / ftol / maxiter rules (Sec. 2.4 and its est.stat report). */
enum {
    MNL_STOP_NONE = 0,         /* a step was taken, no rule met (newton_step) */
    MNL_STOP_GTOL = 1,         /* ||g||_2 <= gtol                          */
    MNL_STOP_FTOL = 2,         /* |l_new - l_old| < ftol                   */
    MNL_STOP_MAXITER = 3,      /* iteration cap reached                    */
    MNL_STOP_LS_FAIL = 4,      /* no halving raised l; theta unchanged     */
    MNL_STOP_NOT_PD = 5,       /* Cholesky pivot at or below round-off     */
    MNL_STOP_NONFINITE = 6     /* l or g not finite                        */
};

/* Arithmetic of the Hessian contraction (Eq. 10).  The log-likelihood,
 * gradient, Cholesky solve and line search are FP64 in every mode, so the
 * fixed point g(theta) = 0 does not depend on this choice; a rounded Hessian
 * only changes the convergence rate of the iteration. */
typedef enum {
    MNL_PREC_FP64 = 0,         /* FP64 MFMA, FP64 accumulation            */
    MNL_PREC_FP32 = 1,         /* FP32 operands on MFMA, FP32 accumulation */
    MNL_PREC_BF16 = 2          /* BF16 operands on MFMA, FP32 accumulation */
} mnl_prec;

/* One fitting problem (Sec. 3.1 notation). */
typedef struct {
    int64_t N;                 /* individuals, >= 1                        */
    int32_t K;                 /* alternatives, >= 2 (K = 2: binary logit) */
    int32_t p;                 /* columns of X (intercept included), >= 0  */
    int32_t g;                 /* generic-coefficient variables, >= 0      */
    int32_t a;                 /* alternative-specific-coef vars, >= 0     */
    const double *X;           /* [N][p]; may be NULL iff p == 0           */
    const double *Y;           /* [N][K][g]; may be NULL iff g == 0        */
    const double *Z;           /* [N][K][a]; may be NULL iff a == 0        */
    const int32_t *choice;     /* [N] observed alternative, 0..K-1         */
    const double *w;           /* [N] frequency weights >= 0, NULL = ones  */
} mnl_problem;

/* Newton direction.  NEWTON solves H delta = -g exactly by factoring H
 * (Eq. 6).  NEWTON_CG is the inexact (truncated) Newton method the paper
 * names as its next step (Sec. 5): conjugate gradients on (-H) d = g from
 * d = 0 with FP64 Hessian-vector products (H is never formed), stopped at
 * relative residual min(1/2, sqrt(||g||_2 / ||g_0||_2)), g_0 the gradient
 * where the call started (so a single newton_step uses 1/2), after
 * cg_maxiter products, or
 * at a direction of non-positive curvature (d = g if that is the first);
 * the line search and stop rules are Newton's.  prec does not apply. */
typedef enum {
    MNL_METHOD_NEWTON = 0,
    MNL_METHOD_NEWTON_CG = 1
} mnl_method;

/* Fit options; defaults (mnl_default_opts) are mnlogit's maxiter = 50,
 * ftol = 1e-6, gtol = 1e-6 (Sec. 2.4), FP64 Hessian, 30 halvings, a
 * line-search acceptance slack of 64 ulps of |l|, no validation, and the
 * exact Newton direction (cg_maxiter 250 when NEWTON_CG is chosen). */
typedef struct {
    int32_t maxiter;           /* >= 0                                     */
    double ftol;               /* stop when |dl| < ftol (0 disables)       */
    double gtol;               /* stop when ||g||_2 <= gtol                */
    int32_t prec;              /* mnl_prec of the Hessian                  */
    int32_t ls_max;            /* halvings before MNL_STOP_LS_FAIL, >= 0   */
    double ls_tol_ulps;        /* accept l_t >= l - ls_tol_ulps*eps*|l|    */
    int32_t validate;          /* nonzero: check choices and finiteness of
                                  the data before fitting                  */
    int32_t method;            /* mnl_method of the Newton direction       */
    int32_t cg_maxiter;        /* NEWTON_CG: Hessian-vector products per
                                  iteration at most, >= 1                  */
    int32_t graph;             /* > 0: from the second iteration on, each
                                  Newton step (Hessian, factorisation,
                                  full-step trial) is captured once per
                                  parity of the alternating buffers into a
                                  HIP graph and replayed; 0: eager steps;
                                  < 0 (MNL_GRAPH_AUTO, the default): graph
                                  steps for n_p <= MNL_GRAPH_AUTO_MAX_NP,
                                  where launches dominate a step.  Needs a
                                  non-default stream; NEWTON_CG, n_p >=
                                  2048, the default stream and
                                  mnl_newton_step run eagerly.  Growth of
                                  the workspace (the first FP64 retry of a
                                  mixed Hessian) drops the captured steps,
                                  which are captured again.  Results are
                                  bitwise the same.                        */
} mnl_fit_opts;

#define MNL_GRAPH_AUTO (-1)
#define MNL_GRAPH_AUTO_MAX_NP 512

/* Report of a fit or of one Newton step (mnlogit's est.stat). Times in ms:
 * t_* are host wall times of the phases; t_hess_kernel and t_pass_kernel
 * are GPU times (HIP events on the caller's stream) of the Hessian MFMA
 * kernel and of the fused pass kernel, summed over n_hess / n_pass
 * launches. */
typedef struct {
    int32_t iters;             /* Newton iterations taken                  */
    int32_t ls_iters;          /* line-search trial evaluations            */
    int32_t ls_backtracks;     /* halvings (trials beyond the full step)   */
    int32_t stop_reason;       /* MNL_STOP_*                               */
    int32_t hess_fallbacks;    /* mixed precision: Hessians recomputed in
                                  FP64 after a failed factorisation       */
    int32_t n_hess;            /* Hessian formations                       */
    double loglik;             /* l at the returned theta                  */
    double grad_norm;          /* ||g||_2 at the returned theta (fit), at
                                  the input theta (newton_step)            */
    double loglik_diff;        /* l change of the last step                */
    double t_total;            /* wall time of the call                    */
    double t_loglik_grad;      /* first pass (l, g, P) before stepping     */
    double t_hessian;          /* Hessian formation (NEWTON_CG: the inner
                                  conjugate-gradient solve)                */
    double t_chol;             /* Cholesky factorisation + solves (0 for
                                  NEWTON_CG)                               */
    double t_ls;               /* line-search passes                       */
    double t_hess_kernel;      /* GPU time in the Hessian MFMA kernel      */
    double t_pass_kernel;      /* GPU time in the fused pass kernel        */
    int32_t n_pass;            /* fused passes run                         */
    int32_t cg_iters;          /* NEWTON_CG: Hessian-vector products       */
    int32_t graph_steps;       /* Newton steps run as graph replays (their
                                  kernels are not in t_hess_kernel, n_hess,
                                  t_pass_kernel, n_pass)                   */
    int32_t reserved;
} mnl_fit_info;

/* Library version string ("major.minor"). */
const char *mnl_version(void);

/* Static name of a return code. */
const char *mnl_strerror(int code);

/* Fill *opts with the defaults above.  opts must not be NULL. */
void mnl_default_opts(mnl_fit_opts *opts);

/* n_p = (K-1) p + K a + g (Eq. 8), or -1 for K < 2 or negative sizes. */
int64_t mnl_num_params(int32_t K, int32_t p, int32_t g, int32_t a);

/* Create a context on HIP device `device`.  *ctx receives the handle.
 * The library owns the context's device workspace and grows it on demand;
 * workspace_bytes caps it: a call that would grow the workspace past that
 * many bytes fails with MNL_ERR_OOM (the same as a failed device
 * allocation) and the workspace keeps what it held.  0: no cap.  The cap
 * covers the workspace (mnl_workspace_bytes), not the small per-shape plan
 * tables.  Returns MNL_ERR_ARG for ctx == NULL or an invalid device,
 * MNL_ERR_HIP if the device cannot be selected. */
int mnl_create(mnl_ctx **ctx, int device, size_t workspace_bytes);

/* Free the context and its workspace (NULL is ignored).  Waits for the
 * context's outstanding work. */
void mnl_destroy(mnl_ctx *ctx);

/* Bytes of device workspace currently held by the context. */
size_t mnl_workspace_bytes(const mnl_ctx *ctx);

/* Last error message of the context (empty string if none). */
const char *mnl_last_error(const mnl_ctx *ctx);

/* Log-likelihood and gradient at theta (Eqs. 2-5 and 9), one fused pass.
 *   theta   [n_p] device, input.
 *   loglik  [1] device, output: weighted log-likelihood (Eq. 5).
 *   grad    [n_p] device, output, may be NULL: dl/dtheta in Eq. 8 layout.
 *   P       [N][K] device, output, may be NULL: choice probabilities
 *           (Eqs. 3-4), alternative 0 in column 0.
 * Asynchronous on `stream`. */
int mnl_loglik_grad(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                    double *loglik, double *grad, double *P, void *stream);

/* mnl_loglik_grad for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, bitwise, with no hipMalloc,
 * hipFree or allocating library call.  Its scratch (the pass's
 * per-workgroup partial rows, n_wg x (n_p + 1) doubles, n_wg <= 768) is a
 * static device buffer of MNL_NOALLOC_SCRATCH_BYTES per GPU, held from the
 * library's load until the process ends; shapes needing more return
 * MNL_ERR_UNSUPPORTED before anything is enqueued.  Every call on one GPU
 * shares that buffer: calls that overlap on one device (other streams,
 * other contexts or threads) race and must be ordered by the caller.
 * Arguments and layouts as for mnl_loglik_grad; the context is only read
 * (its device and its error message). */
#define MNL_NOALLOC_SCRATCH_BYTES (32u << 20)
int mnl_loglik_grad_noalloc(mnl_ctx *ctx, const mnl_problem *prob,
                            const double *theta, double *loglik, double *grad,
                            double *P, void *stream);

/* Full Hessian at theta (Eq. 10), Hessian sign (negative semidefinite).
 *   theta   [n_p] device, input.
 *   prec    mnl_prec of the contraction.
 *   H       [n_p][n_p] device, output, full symmetric matrix.
 * Asynchronous on `stream`. */
int mnl_hessian(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                int32_t prec, double *H, void *stream);

/* One Newton-Raphson iteration from theta (Eq. 6 with the halving line
 * search).  If ||g(theta)||_2 <= opts->gtol no step is taken and
 * step->stop_reason = MNL_STOP_GTOL.  Otherwise theta is replaced by the
 * accepted trial theta + t delta, delta = -H^{-1} g, and stop_reason is
 * MNL_STOP_NONE, or NOT_PD / LS_FAIL / NONFINITE with theta unchanged.
 *   theta   [n_p] device, input and output.
 *   opts    host, NULL = defaults.
 *   step    host, output.
 * Synchronises `stream`. */
int mnl_newton_step(mnl_ctx *ctx, const mnl_problem *prob, double *theta,
                    const mnl_fit_opts *opts, mnl_fit_info *step,
                    void *stream);

/* Newton-Raphson fit (Sec. 3.1): iterate until ||g||_2 <= gtol (checked at
 * the top of each iteration), |dl| < ftol (after a step) or maxiter.
 *   theta0     [n_p] device start, NULL = zeros (mnlogit's start = NULL).
 *   theta_out  [n_p] device, output (may equal theta0).
 *   opts       host, NULL = defaults.
 *   info       host, output.
 * NOT_PD, LS_FAIL and NONFINITE end the fit with that stop_reason and the
 * last accepted theta; the call still returns MNL_OK.  Synchronises
 * `stream`. */
int mnl_fit(mnl_ctx *ctx, const mnl_problem *prob, const double *theta0,
            const mnl_fit_opts *opts, double *theta_out, mnl_fit_info *info,
            void *stream);

/* Many small Newton-Raphson fits at once (Sec. 3.1: Eqs. 2-6, 9 and 10 and
 * the halving line search, the stop rules of mnl_fit), one workgroup per
 * fit of a persistent kernel that takes fits from a device work list.  A
 * fit's state (theta, gradient, -H and its L D L^T factor) stays on chip
 * for the whole fit; every sum runs in an order fixed by the fit's own
 * shape, so each result is bitwise the same whatever else is in the batch.
 * The arithmetic differs from mnl_fit's kernels in rounding only.
 *   probs      host array [nfits] of problems with DEVICE data.
 *   theta0     host array [nfits] of device [n_p] starts, or NULL (zeros);
 *              a NULL entry is a zero start.
 *   opts       host array [nfits], NULL = defaults for all.  Each must ask
 *              for FP64 Newton steps without validation (prec FP64, method
 *              NEWTON, validate 0; graph and cg_maxiter are ignored), else
 *              MNL_ERR_UNSUPPORTED.
 *   theta_out  host array [nfits] of device [n_p] outputs (may equal the
 *              fit's theta0).
 *   info       host array [nfits], output: iters, ls_iters, ls_backtracks,
 *              stop_reason, n_hess, n_pass, loglik, grad_norm and
 *              loglik_diff as from mnl_fit; t_total is the batch's wall
 *              time; t_loglik_grad, t_hessian, t_chol and t_ls are the
 *              fit's own phases timed on the device's constant-rate clock
 *              by its workgroup; the other times and counters are 0.
 * Shape limits (MNL_ERR_UNSUPPORTED beyond them): K <= 64, g <= 8,
 * n_p <= 128, and the fit's LDS layout (A = -H with row stride n_p | 1,
 * five vectors of n_p, and for 4 observations two staged copies of their
 * p + K a + K g values, weight and choice, and K + g + g (g+1)/2 +
 * (K-1) p + K a per-observation products) within 160 KiB.  Nothing is written for a call that fails its
 * checks.  Not capturable into a HIP graph (host copies of the work
 * list).  Synchronises `stream`. */
int mnl_fit_batch(mnl_ctx *ctx, int32_t nfits, const mnl_problem *probs,
                  const double *const *theta0, const mnl_fit_opts *opts,
                  double *const *theta_out, mnl_fit_info *info,
                  void *stream);

/* 1 if a fit of this shape (sizes only) with these options (NULL =
 * defaults) is one the server runs through mnl_fit_batch: within its
 * limits, FP64 Newton without validation, and N n_p^2 <= MNL_BATCH_MAX_WORK
 * (a fit the size of one workgroup); else 0. */
#define MNL_BATCH_MAX_WORK (((int64_t)1) << 26)
int mnl_batch_eligible(const mnl_problem *shape, const mnl_fit_opts *opts);

/* Hessian-vector product H(theta) v (Eq. 10's H, never formed): one fused
 * pass for P at theta, then one pass of v through -sum_i w_i J_i^T
 * (diag P_i - P_i P_i^T) J_i, J_i = dU_i/dtheta.  prob->choice is not read
 * (may be NULL).
 *   theta, v  [n_p] device, input.
 *   Hv        [n_p] device, output (Hessian sign).
 * Asynchronous on `stream`. */
int mnl_hessvec(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                const double *v, double *Hv, void *stream);

/* ---- Collinearity check (Sec. 2.4 linDepTol, App. B) ---------------------- */

/* Variables to keep so that App. B's necessary conditions for a
 * non-singular Hessian hold: X and every Z_k = Z[:, k, :] of full column
 * rank, and the differenced generic data Y_k - Y_0 (k >= 1) stacked over
 * alternatives of full column rank.  Within each matrix the columns are
 * taken in order and column j is dropped when its part orthogonal to the
 * kept columns before it has norm below tol times its own norm (mnlogit's
 * qr with tol = linDepTol, default 1e-6); a zero column is dropped.  A Z
 * variable dependent in any alternative is dropped for all.  Computed on
 * Gram matrices (one pass over the observations; library GEMMs beyond 4096
 * Gram entries or 8192 doubles per observation), then an ordered
 * elimination on the device, which agrees with QR while the kept columns'
 * condition number squared times eps stays well below tol^2.
 * prob->choice is not read (may be NULL).
 *   tol      in [0, 1).
 *   keep_x   [p] host int32, output: 1 keep, 0 drop (NULL iff p == 0).
 *   keep_y   [g] host int32, output (NULL iff g == 0).
 *   keep_z   [a] host int32, output (NULL iff a == 0).
 * At most 1024 columns per kind (MNL_ERR_UNSUPPORTED).  On the library
 * route the workspace also takes N (K-1) g doubles for the differenced
 * data.  Synchronises `stream`. */
int mnl_collinear(mnl_ctx *ctx, const mnl_problem *prob, double tol,
                  int32_t *keep_x, int32_t *keep_y, int32_t *keep_z,
                  void *stream);

/* Copies of the data with only the kept columns (flags as mnl_collinear
 * returns them, host int32):
 *   X_out  [N][p'] device, Y_out [N][K][g'], Z_out [N][K][a'], p', g', a'
 *          the kept counts; an output may be NULL when its count is 0.
 * The reduced problem fits theta' of n_p' = (K-1) p' + K a' + g'
 * coefficients, those of the dropped variables being absent.
 * Asynchronous on `stream` (the selection indices are copied first). */
int mnl_select_columns(mnl_ctx *ctx, const mnl_problem *prob,
                       const int32_t *keep_x, const int32_t *keep_y,
                       const int32_t *keep_z, double *X_out, double *Y_out,
                       double *Z_out, void *stream);

/* ---- Fitted-model methods (Sec. 2.4: summary and predict) ----------------- */

/* Choice probabilities on (new) data at theta: Eqs. 3-4 at the utilities of
 * Eq. 2, one fused pass.  prob->choice and prob->w are not read (either may
 * be NULL).
 *   theta   [n_p] device, input.
 *   P       [N][K] device, output; alternative 0 in column 0.
 * Asynchronous on `stream`. */
int mnl_predict(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                double *P, void *stream);

/* The summary's coefficient table at theta (normally the fitted one): the
 * asymptotic standard errors se = sqrt(diag((-H)^{-1})), H the FP64 Hessian
 * of Eq. 10 at theta, the Wald statistics z = theta / se and their two-sided
 * normal p-values erfc(|z| / sqrt 2).  One FP64 Hessian and one LDL^T
 * factorisation of -H with n_p identity rows appended (the workspace holds
 * (2 n_p + 1) x n_p doubles).  prob->choice is not read (may be NULL).
 *   theta   [n_p] device, input.
 *   se      [n_p] device, output.
 *   zval    [n_p] device, output, may be NULL.
 *   pval    [n_p] device, output, may be NULL.
 * MNL_ERR_NOT_PD (outputs unspecified) when -H has a pivot at or below
 * n_p * eps * max_k(-H_kk).  Synchronises `stream`. */
int mnl_stderr(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
               double *se, double *zval, double *pval, void *stream);

/* ---- Hypothesis tests (Sec. 2.4: lrtest, waldtest, scoretest, hmftest) ---
 * The statistics are quadratic forms in the estimate's covariance or the
 * Hessian; these three calls supply them (the likelihood ratio needs only
 * the two fits' log-likelihoods). */

/* Covariance of the estimate, (-H)^{-1} at theta (FP64 Hessian of Eq. 10),
 * restricted to the coefficients idx:
 *   idx   [nidx] host int32, coefficient indices in Eq. 8 order; NULL with
 *         nidx == 0 means all n_p coefficients in order.
 *   V     [s][s] device, output, s = nidx (or n_p); V[a][b] =
 *         ((-H)^{-1})[idx[a]][idx[b]], exactly symmetric.
 * One FP64 Hessian and one factorisation with identity rows (as
 * mnl_stderr).  MNL_ERR_NOT_PD when -H fails the pivot test; MNL_ERR_ARG
 * for an index outside [0, n_p).  prob->choice is not read.  Synchronises
 * `stream`. */
int mnl_covariance(mnl_ctx *ctx, const mnl_problem *prob, const double *theta,
                   const int32_t *idx, int32_t nidx, double *V,
                   void *stream);

/* Quadratic form d^T M^{-1} d with M = A - B and d = x - x0 (B and x0
 * optional) for a symmetric positive definite M, through M's L D L^T
 * factor (d rides along as an extra row: sum_k y_k^2 D_k with
 * y = D^{-1} L^{-1} d).  With hessian_sign != 0, M is negative definite
 * (a Hessian as mnl_hessian returns it) and the form is d^T (-M)^{-1} d:
 * the score statistic for M = H, d = g.  The Wald statistic is
 * theta_S^T V_SS^{-1} theta_S; the Hausman-McFadden statistic takes
 * A = V_subset, B = V_full, x = theta_subset, x0 = theta_full.
 *   A, B   [n][n] device, inputs (not modified; lower triangles read).
 *   x, x0  [n] device, inputs.
 *   out    host, output.
 * MNL_ERR_NOT_PD when a pivot is at or below n eps max_k M_kk.
 * Synchronises `stream`. */
int mnl_quadform(mnl_ctx *ctx, const double *A, const double *B,
                 const double *x, const double *x0, int64_t n,
                 int32_t hessian_sign, double *out, void *stream);

/* Upper tail P(chi^2_df > x) of the chi-square distribution (host):
 * the p-value of the test statistics above.  NaN for df <= 0. */
double mnl_chi2_sf(double x, double df);

/* Likelihood-ratio statistic of nested fits (host): *stat =
 * 2 (loglik_full - loglik_restricted) and, when pval is not NULL, its
 * chi-square tail with df degrees of freedom (the number of restrictions).
 * MNL_ERR_ARG for df <= 0 or a NULL stat. */
int mnl_lrtest(double loglik_full, double loglik_restricted, int32_t df,
               double *stat, double *pval);

/* ---- Serving: continuous batching of independent fits -------------------
 *
 * A server runs many fits at once on one device.  Requests arrive with
 * their data in HOST memory; each is admitted, in arrival order, as soon as
 * a slot is free and its device footprint (mnl_fit_footprint) fits in what
 * the HBM budget has left, so requests that arrive while others are on the
 * GPU join the running mix.  An admitted fit copies its data to the device
 * and keeps all of its state there (data, P, H, workspace) until it ends;
 * each slot runs its fit on a HIP stream of its own, so the fits' kernels
 * overlap on the device.  Every fit's reductions use partitions fixed by
 * its own shape, so its result is bitwise the same alone and in any mix.
 * Small fits run together: a slot that admits a request the batched
 * kernel takes (mnl_batch_eligible) also admits the eligible requests
 * queued right behind it, in arrival order, up to max_group and the
 * budget, and runs the group as one mnl_fit_batch; such a request's
 * result is bitwise the same as mnl_fit_batch of it alone (the other
 * requests run through mnl_fit's path, bitwise the same as mnl_fit).
 * A request whose footprint exceeds the whole budget is refused at submit.
 * Device memory comes from a stream-ordered pool owned by the server; the
 * budget bounds the bytes that admitted fits have requested from it.
 */
typedef struct mnl_server mnl_server;

typedef struct {
    int32_t device;            /* HIP device                               */
    int32_t slots;             /* fits in flight at once, 1..256            */
    size_t hbm_budget;         /* bytes admitted fits may hold; 0 = 80 % of
                                  the device memory free at creation       */
    int32_t host_only;         /* nonzero: scheduler test mode with no
                                  device: admission, slots and accounting
                                  as usual, but an admitted request only
                                  waits host_fit_ms and returns theta = 0
                                  (stop_reason MNL_STOP_NONE, no
                                  iterations); hbm_budget must be > 0      */
    int32_t max_group;         /* most requests one slot runs together
                                  through mnl_fit_batch; 0 = 1024, 1 = one
                                  request per slot, >= 0                   */
    double host_fit_ms;        /* host_only: time each "fit" (or group of
                                  fits) takes                              */
} mnl_server_opts;

/* One finished request (mnl_server_wait).  Times in ms on the server clock
 * (mnl_server_now_ms): t_arrival as given at submit, t_admit when a slot
 * took it, t_done when theta was in host memory.  Latency is t_done -
 * t_arrival (queueing, host-to-device copies and the fit). */
typedef struct {
    int64_t id;                /* from mnl_server_submit                   */
    int32_t status;            /* MNL_OK or the MNL_ERR_* of the fit        */
    int32_t slot;              /* slot that ran it                          */
    double t_arrival, t_admit, t_done;
    size_t footprint;          /* device bytes reserved for it              */
    mnl_fit_info info;         /* as from mnl_fit                           */
} mnl_server_result;

/* Counters of a server (mnl_server_stats). */
typedef struct {
    int64_t submitted, completed;
    int32_t queued, running;
    int32_t max_running;       /* most fits in flight at one time           */
    int32_t reserved;
    size_t budget, in_use, peak_in_use; /* footprint bytes                 */
} mnl_server_stats;

/* Device bytes a fit of this shape holds while it runs: its data copy plus
 * the library's workspace (an upper bound).  Only the sizes (N, K, p, g,
 * a) and whether w is NULL are read.  Returns -1 for an invalid shape. */
int64_t mnl_fit_footprint(const mnl_problem *shape, int32_t prec);

/* Milliseconds on the server clock (a monotonic host clock). */
double mnl_server_now_ms(void);

/* Create a server and its slot threads.  Returns MNL_ERR_ARG for bad
 * options, MNL_ERR_HIP / MNL_ERR_OOM if streams or the pool fail. */
int mnl_server_create(mnl_server **srv, const mnl_server_opts *opts);

/* Stop the server: queued requests that were not admitted are dropped
 * (never reported), running fits finish, then all resources are freed.
 * NULL is ignored. */
void mnl_server_destroy(mnl_server *srv);

/* Queue a fit.
 *   prob       host struct whose array pointers are HOST memory (page-
 *              locked memory makes the copies faster); the arrays must stay
 *              valid and unchanged until the request's result is returned
 *              by mnl_server_wait.
 *   theta0     host [n_p] start or NULL (zeros); same lifetime rule.
 *   opts       fit options (copied), NULL = defaults.
 *   theta_out  host [n_p], written before the result is reported.
 *   t_arrival  arrival time on the server clock; < 0 means now.
 *   id         receives the request id (>= 0).
 * Returns MNL_ERR_ARG for an invalid problem or options and MNL_ERR_OOM if
 * the footprint exceeds the whole budget; nothing is queued then. */
int mnl_server_submit(mnl_server *srv, const mnl_problem *prob,
                      const double *theta0, const mnl_fit_opts *opts,
                      double *theta_out, double t_arrival, int64_t *id);

/* Move up to max_results finished requests into out[] (completion order)
 * and set *n_out.  Blocks until at least one is available or timeout_ms has
 * passed (0 = do not block, < 0 = no limit). */
int mnl_server_wait(mnl_server *srv, mnl_server_result *out,
                    int32_t max_results, double timeout_ms, int32_t *n_out);

/* Snapshot of the server's counters. */
int mnl_server_get_stats(mnl_server *srv, mnl_server_stats *st);

#ifdef __cplusplus
}
#endif

#endif /* MNL_H */
