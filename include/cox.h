/*
 * cox.h -- C ABI of libcoxhip: l1-regularised Cox proportional-hazards
 * regression by proximal gradient (ISTA) on one AMD Instinct MI355X (gfx950).
 *
 * The problem (Ko, Zhou, Zhou and Won, "DistStat.jl", Section 5.3): subjects
 * i = 1..n with covariate row x_i (p SNPs), observed time y_i = min(t_i, c_i)
 * and event indicator delta_i.  The Breslow log partial likelihood is
 *     L(beta) = sum_i delta_i [ eta_i - log sum_{j: y_j >= y_i} exp(eta_j) ],
 *     eta = X~ beta,
 * (ties share their risk set, Breslow's convention of Section 6), and the
 * library minimises  f_lambda(beta) = -L(beta) + lambda ||beta||_1,  the
 * minimisation form of the paper's "maximise L - lambda ||beta||_1", with the
 * iteration of Section 5.3:
 *     w = exp(eta),  W_j = sum_{i: y_i >= y_j} w_i,
 *     r = (I - P) delta,  P_ij = 1(y_i >= y_j) w_i / W_j,
 *     beta <- S_{sigma lambda}(beta + sigma X~' r)
 * where S is the soft-thresholding operator of Section 4.2 and sigma the step.
 * (The paper writes the threshold as lambda; the threshold of the proximal map
 * of sigma * lambda ||.||_1 is sigma * lambda, which is what is used here.)
 *
 * Covariates and penalty factors (Section 6's application, where sex and the
 * top principal components enter the model unpenalised beside the SNPs).  A
 * dense FP32 block Z of q covariates may be attached (cox_set_covariates); the
 * model matrix is then [X~ | Z] and every coefficient vector has
 * ptot = p + q entries, the covariates last.  Each column j has a penalty
 * factor pf_j >= 0 (cox_set_penalty_factors; by default 1 for the columns of
 * X and 0 for the covariates): the objective is
 *     f_lambda(beta) = -L(beta) + lambda sum_j pf_j |beta_j|
 * and the step's threshold for column j is sigma * lambda * pf_j, so a column
 * with pf_j = 0 is unpenalised.
 *
 * Data layout.  X is dense, column-major (each SNP column contiguous), n rows
 * by p columns with leading dimension ldx >= n, the column split of Section
 * 4.1.  X~ is X itself for COX_X_F32.  For the 1-byte genotype types X holds
 * allele counts g and X~_ij = (g_ij - col_center[j]) * col_scale[j] is formed
 * on the fly (NULL center = 0, NULL scale = 1).  Vectors for B coefficient
 * vectors are stored b-major: beta[b*ptot + j] (ptot = p without covariates),
 * eta[b*n + i].
 *
 * Conventions shared by every entry point.
 *  - Return value: a cox_status.  No C++ exception or abort crosses the ABI.
 *  - Argument errors are detected before any device work and leave outputs and
 *    the context untouched (COX_ERR_INVALID_ARG).
 *  - Padding: for the 1-byte types with ldx a multiple of 16, kernels read whole
 *    16-byte runs, so every column -- the last one included -- must be
 *    allocated up to ldx bytes (rows n..ldx-1 are read and ignored).  A torch
 *    tensor of shape (p, ldx) satisfies this.
 *  - Pointers marked "dev" are device memory of the context's GPU; "host" are
 *    host memory.  The caller owns every buffer it passes.  X, col_center and
 *    col_scale are BORROWED: they must stay valid and unchanged until
 *    cox_destroy; X is never copied.
 *  - All device work is ordered on the stream given to cox_setup.  Entry points
 *    that return host values synchronise that stream before returning;
 *    device outputs are otherwise stream-ordered.
 *  - A context is not thread-safe; use one context per stream.
 *  - Results are deterministic: no floating-point atomics, fixed reduction order.
 */
#ifndef COX_H
#define COX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cox_ctx cox_ctx;

typedef enum {
    COX_OK = 0,
    COX_ERR_INVALID_ARG = 1,   /* bad shape, pointer, time, event, batch size or option */
    COX_ERR_OUT_OF_MEMORY = 2, /* device or host allocation failed; nothing leaked */
    COX_ERR_DEVICE = 3,        /* a HIP runtime call failed */
    COX_ERR_NUMERIC = 4,       /* the loss or the gradient became non-finite */
    COX_ERR_NOT_CONVERGED = 5, /* max_iter reached; outputs are valid */
    COX_ERR_UNSUPPORTED = 6    /* valid request this build does not serve */
} cox_status;

typedef enum {
    COX_X_F32 = 0,      /* float, used as given */
    COX_X_FP8_E4M3 = 1, /* OCP FP8 E4M3 (e4m3fn) codes of the allele counts */
    COX_X_INT8 = 2      /* signed 8-bit allele counts */
} cox_xtype;

typedef struct {
    const void *X;           /* dev, column-major, element (i, j) at X[j*ldx + i]; borrowed */
    int32_t xtype;           /* cox_xtype */
    int64_t n, p, ldx;       /* 1 <= n < 2^31, 1 <= p < 2^31, ldx >= n */
    const float *col_center; /* dev [p] or NULL: genotype centre mu_j; borrowed; 1-byte types only */
    const float *col_scale;  /* dev [p] or NULL: genotype scale s_j (1/SD); borrowed; 1-byte types only */
} cox_matrix;

/* Create a context for one data set (Section 5.3's X, y, delta).
 *   time  host [n], finite observed times y_i; copied.  Subjects are ordered
 *         internally by non-increasing time (stable by index), so the risk-set
 *         sums become cumulative sums (Section 5.3); tied times form Breslow
 *         groups (Section 6).
 *   event host [n], each 0 (censored) or 1 (event); copied.
 *   max_batch  the largest B any later call passes (1..64); sizes the workspace.
 *   hip_stream a hipStream_t (NULL: the default stream).
 * Returns INVALID_ARG (bad X descriptor, ldx < n, non-finite time, event not
 * 0/1, max_batch out of range, NULL pointers), OUT_OF_MEMORY or DEVICE on
 * failure, with *out set to NULL. */
cox_status cox_setup(cox_ctx **out, const cox_matrix *X, const double *time, const int32_t *event,
                     int32_t max_batch, void *hip_stream);

/* Free the context's workspace.  NULL is accepted. */
cox_status cox_destroy(cox_ctx *ctx);

/* Static text for a status code. */
const char *cox_status_string(cox_status s);

/* Human-readable detail of the last error on ctx (empty if none), NUL-terminated
 * into buf[len].  INVALID_ARG if ctx or buf is NULL or len is 0. */
cox_status cox_last_error(const cox_ctx *ctx, char *buf, size_t len);

/* Value and gradient of the NEGATIVE log partial likelihood, -L(beta_b), for B
 * coefficient vectors (Section 5.3: the gradient of L is X~'(I - P) delta).
 *   beta  dev [B][ptot] float
 *   loss  host [B] double: -L(beta_b)
 *   grad  dev [B][ptot] float, or NULL for the loss only: -[X~ Z]' r_b
 * eta = X~ beta_b is formed to FP64 accuracy: by FP64 passes of up to 8 vectors,
 * or, for B > 8 over one-byte allele counts, by three exact 22-bit integer
 * passes on the matrix cores (whatever the first pass leaves of each vector is
 * taken by the next; at most 2^-69 max|beta_b| per coefficient is left over).
 * NUMERIC if a loss is non-finite (e.g. NaN in beta). Synchronises. */
cox_status cox_loss_grad(cox_ctx *ctx, const float *beta, int32_t B, double *loss, float *grad);

/* One proximal-gradient (ISTA) step in place for each b (Section 5.3):
 *   beta_bj <- S_{step*lambda_b*pf_j}(beta_bj + step * ([X~ Z]' r_b)_j)
 *   beta        dev [B][ptot] float, in/out
 *   lambdas     host [B], each >= 0 and finite
 *   step        sigma > 0
 *   obj_before  host [B] or NULL: f_lambda_b(beta_b) before the step.
 * Synchronises when obj_before is not NULL. */
cox_status cox_prox_step(cox_ctx *ctx, float *beta, int32_t B, const double *lambdas, double step,
                         double *obj_before);

/* Apply the soft-threshold update alone (the elementwise kernel), given a
 * gradient of the negative log likelihood.  This is the proximal half of the
 * iteration of Section 5.3 with the soft-thresholding operator of Section 4.2
 * (threshold step * lambda, as in cox_prox_step):
 *   beta_bj <- S_{step*lambda_b*pf_j}(beta_bj - step * grad_bj)
 *   beta dev [B][ptot] in/out; grad dev [B][ptot]; lambdas host [B] >= 0; step > 0. */
cox_status cox_prox_apply(cox_ctx *ctx, float *beta, const float *grad, int32_t B, const double *lambdas,
                          double step);

typedef struct {
    int32_t max_iter;   /* >= 0: the largest number of steps for each b */
    double tol;         /* >= 0: stop b when |f_k - f_{k-lag}| / (|f_k| + 1) < tol (Section 6); 0: never */
    int32_t lag;        /* 1..32; the paper uses 10 */
    double step;        /* > 0: sigma; <= 0: 1 / (2 ||X~||_2^2) from cox_opnorm2 (Section 5.3) */
    int32_t warm_start; /* 0: start from beta = 0; 1: start from the beta passed in (FP32; eta is formed
                           afresh by a dense pass); 2: resume -- continue the last cox_fit_path on this
                           context from its own FP64 iterate, accumulated eta and stopping-rule history,
                           so that K1 steps and a resume to max_iter = K2 give bit for bit the results
                           of one call with max_iter = K2.  Resuming needs the same B, lambdas, step
                           (<= 0: the last call's), eta_mode, residual_bits and covariates, max_iter at
                           least the last call's, and no other call on the context in between that
                           uses its workspace (INVALID_ARG otherwise; UNSUPPORTED with persistent).
                           Lambdas that had converged stay as they were; beta is output only; the
                           trace holds NaN for the steps of the earlier call. */
    int32_t persistent; /* 0: one launch per phase of each step, the host checking the stopping flags
                           every `poll` steps; 1: the whole call -- every step of every b, the stopping
                           rule included -- in one persistent (cooperative) launch whose workgroups are
                           all resident at once, with grid-wide barriers between the phases.
                           persistent = 1 serves the vector path: B <= 8 (not the batched matrix-core
                           pass), eta_mode 0, no covariate block, X 16-byte aligned with ldx times the
                           element size a multiple of 16; other requests return UNSUPPORTED before any
                           device work.  Both forms run the same per-workgroup code in the same order
                           and give bit-identical results.  A barrier that waits longer than 60 s
                           abandons the launch (DEVICE). */
    int32_t deterministic; /* 0 or 1.  Results are always bit-reproducible run to run (fixed-order
                              reductions, no floating-point atomics), so both values give the same
                              computation; 1 documents the requirement. */
    int32_t eta_mode;   /* 0: eta updated from the columns whose beta changed (FP64 accumulator);
                           1: eta recomputed every step by a dense product (as in cox_loss_grad: FP64
                           passes of up to 8 vectors, or three exact limb passes on the matrix cores
                           for B > 8 over allele counts) */
    int32_t poll;       /* steps between host checks of the convergence flags; <= 0: 16 */
    int32_t residual_bits; /* batched matrix-core gradient pass only (allele counts, B > 8): the
                              residual r_b is rounded to integers |R| <= 2^bits relative to
                              max |r_b| before the exact int8 contraction.  0 or 22: three
                              limbs (default); 14: two limbs, a third less limb traffic and
                              matrix-core work at about 2^-15 relative rounding of r.  Other
                              values are INVALID_ARG. */
    double *trace;      /* host [B][max_iter + 1] or NULL: trace[b*(max_iter+1) + k] = f_lambda_b(beta_k),
                           the objective at step k of b as the stopping rule saw it, for k = 0..k_b;
                           entries past k_b are NaN */
} cox_fit_opts;

/* Solve B problems (one per lambda_b) by ISTA, all sharing each pass over X.
 * For each b, from beta_0 (0, or the input when warm_start): at step k the
 * objective f_k = f_lambda_b(beta_k) is evaluated; b stops at the first k with
 * k >= lag and |f_k - f_{k-lag}| / (|f_k| + 1) < tol, or at k = max_iter; else
 * beta_{k+1,j} = S_{sigma lambda_b pf_j}(beta_kj + sigma ([X~ Z]' r)_j).
 *   lambdas host [B] >= 0; opts host (NULL: max_iter 1000, tol 1e-5, lag 10,
 *           step from cox_opnorm2, cold start, not persistent, eta_mode 0, poll 16,
 *           no trace)
 *   beta  dev [B][ptot] float: the start if warm_start, and the result beta_{k_b}
 *   iters host [B] or NULL: k_b, the number of steps taken
 *   obj   host [B] or NULL: f_lambda_b(beta_{k_b})
 * Returns OK when every b met the tolerance, NOT_CONVERGED (outputs valid) when
 * some b reached max_iter, NUMERIC on a non-finite objective.  Synchronises. */
cox_status cox_fit_path(cox_ctx *ctx, const double *lambdas, int32_t B, const cox_fit_opts *opts, float *beta,
                        int32_t *iters, double *obj);

/* lambda_max: the smallest lambda at which every penalised coefficient is zero
 * at the optimum (the top of Section 6's lambda grid; from the optimality
 * condition of the objective of Section 5.3, beta = 0 is optimal exactly when
 * |(X~' r(0))_j| <= lambda pf_j for every j, with r(0) the residual
 * (I - P) delta of Section 5.3 at beta = 0).  With no unpenalised column it is
 * max_j |(X~' r(0))_j| / pf_j,
 * where at beta = 0 every w_i = 1 and r is delta minus the Breslow cumulative
 * hazard.  When some covariates have pf = 0 it is the same maximum over the
 * penalised columns at the unpenalised optimum over those covariates (every
 * other coefficient zero); that optimum is found by ISTA over Z alone with step
 * 1/(2 ||Z||_2^2) until the largest free-covariate gradient is below 1e-10 of
 * its value at zero (at most 100000 steps: NOT_CONVERGED, value still written).
 * An unpenalised column of X (pf_j = 0, j < p) is UNSUPPORTED here (it would
 * need a pass over X per step); fits with one are fine.
 *   lambda_max host [1].  Synchronises. */
cox_status cox_lambda_max(cox_ctx *ctx, double *lambda_max);

/* ||[X~ Z]||_2^2 (||X~||_2^2 without covariates) by power iteration on
 * [X~ Z]'[X~ Z] (Section 4.3, opnorm(X, 2; method = "power"); the paper's
 * defaults are tol 1e-6, maxiter 1000, seed 95376).  Start vector: ptot
 * entries uniform on [-1, 1) from SplitMix64 seeded with `seed` (top 53 bits
 * of each output), normalised.  Stops when the
 * estimate changes by less than tol relative to itself.  Centring is exact.
 *   s2 host [1]; iters host [1] or NULL.  Synchronises. */
cox_status cox_opnorm2(cox_ctx *ctx, double tol, int32_t maxiter, uint64_t seed, double *s2, int32_t *iters);

/* The paper's sequential protocol (Section 6): one lambda after another, each
 * solved to the stopping rule from the previous lambda's solution.
 *   lambdas   host [L] >= 0, in the order solved (typically decreasing)
 *   opts      as cox_fit_path (NULL: its defaults); a step <= 0 is computed once
 *             for the whole sequence.  warm_start applies to the first lambda;
 *             a trace, when given, is host [L][max_iter + 1], row l for lambdas[l].
 *   beta_path dev [L][ptot] float: row l is the solution at lambdas[l] (row 0 is
 *             also the start when warm_start)
 *   iters, obj host [L] or NULL: steps taken and final objective per lambda
 * Returns OK, NOT_CONVERGED (every row valid) when some lambda reached max_iter,
 * or the first other error.  Synchronises. */
cox_status cox_fit_sequence(cox_ctx *ctx, const double *lambdas, int32_t L, const cox_fit_opts *opts,
                            float *beta_path, int32_t *iters, double *obj);

/* Attach the dense block Z of q unpenalised covariates (Section 6's
 * application) beside X: dev float, column-major n x q, element (i, k) at
 * Z[k*ldz + i], ldz >= n; BORROWED (valid and unchanged while the context
 * uses it).  From then on every coefficient and gradient argument has
 * ptot = p + q entries per vector, the covariates last, and the covariates'
 * penalty factors are 0 until cox_set_penalty_factors says otherwise.  q = 0
 * (Z may be NULL) removes the block.  The workspace is sized at cox_setup, so
 * this allocates nothing.  INVALID_ARG for q outside 0..COX_MAX_COVARIATES, a
 * NULL Z with q > 0, or ldz < n.  Synchronises. */
#define COX_MAX_COVARIATES 64
cox_status cox_set_covariates(cox_ctx *ctx, const float *Z, int64_t q, int64_t ldz);

/* Penalty factors of the ptot columns (host [ptot], copied; each finite and
 * >= 0): the objective becomes -L + lambda sum_j pf_j |beta_j| and the threshold
 * of column j sigma * lambda * pf_j.  NULL restores the defaults (1 for the
 * columns of X, 0 for the covariates).  Attaching or removing covariates
 * resets the covariates' factors to 0 and keeps those of X.  Synchronises. */
cox_status cox_set_penalty_factors(cox_ctx *ctx, const double *pf);

/* Post-selection (Section 6): rank the columns a lasso path selects, refit the
 * unpenalised model on them with the covariates, and test each by Wald's test.
 *
 * cox_rank_path: for a path of L solutions (dev [L][ptot] float, row l at the
 * l-th lambda of a decreasing sequence, e.g. from cox_fit_sequence), each
 * column j < p of X gets entry[j] = the first row where it is nonzero (-1:
 * never) and entry_coef[j] = |beta| there (host [p] each; entry_coef
 * nullable).  order (host [p], nullable) receives the entered columns ranked as
 * in Section 6: by entry (the largest lambda first), ties by |coef| at entry
 * (larger first), then by index; *n_entered (nullable) their number.
 * Synchronises. */
cox_status cox_rank_path(cox_ctx *ctx, const float *path, int32_t L, int32_t *entry, float *entry_coef,
                         int64_t *order, int64_t *n_entered);

/* cox_rank_path_noalloc: cox_rank_path for callers that cannot allocate
 * memory (code under HIP graph capture, serving loops, harnesses that forbid
 * hipMalloc).  The same computation and the same outputs as cox_rank_path,
 * bit for bit, but it calls no hipMalloc, hipFree or other allocating routine:
 * its device working memory is a static array inside the library (8 bytes per
 * column, COX_NOALLOC_MAX_COLS columns: 16 MiB, held on each GPU the library
 * runs on until the process ends; its device address is looked up once per
 * GPU, by cox_setup).  Differences: entry_coef must not be NULL (the ranking's
 * tie-break reads it; there is no buffer to hold it otherwise), and p above
 * COX_NOALLOC_MAX_COLS returns UNSUPPORTED before any device work.  Every call
 * on one GPU shares the array: calls that overlap on one GPU (from several
 * threads or streams, before the earlier one returned) race and give wrong
 * results; calls in sequence are safe (each writes every entry it reads).
 * Synchronises. */
#define COX_NOALLOC_MAX_COLS 2097152
cox_status cox_rank_path_noalloc(cox_ctx *ctx, const float *path, int32_t L, int32_t *entry, float *entry_coef,
                                 int64_t *order, int64_t *n_entered);

/* cox_refit: maximum partial likelihood (no penalty) over the m chosen columns
 * of X (cols host [m], distinct, each < p; X~ standardised as everywhere) and
 * all q attached covariates, every other coefficient zero, by Newton's method
 * with the exact Breslow Hessian: each step solves (-H) d = g and halves d
 * until L does not fall (the full step is taken once its predicted gain g'd is
 * at the rounding level of L); it stops when max |g| <= gtol.  The M = m + q
 * columns are gathered once into a dense FP32 block (allocated for the call).
 *   coef  host [M] double: the start (e.g. zeros, or the lasso's values) and the
 *         result, the chosen columns first in the order given, then the
 *         covariates
 *   se    host [M] or NULL: standard errors sqrt(diag((-H)^{-1})) at the result
 *   pval  host [M] or NULL: two-sided Wald p-values erfc(|coef / se| / sqrt 2);
 *         Section 6 keeps a column when pval < alpha / (number tested)
 *   loglik host [1] or NULL: L at the result; iters host [1] or NULL: steps
 *   opts  NULL: 50 steps, gtol 1e-8
 * INVALID_ARG for M outside 1..COX_MAX_REFIT, repeated or out-of-range columns,
 * a non-finite start; NUMERIC when -H is not positive definite (e.g. a constant
 * or repeated column) or L is not finite; NOT_CONVERGED (outputs valid) when
 * max_iter steps end with max |g| > gtol.  Synchronises. */
#define COX_MAX_REFIT 1024
typedef struct {
    int32_t max_iter; /* >= 0 */
    double gtol;      /* >= 0 */
} cox_refit_opts;
cox_status cox_refit(cox_ctx *ctx, const int64_t *cols, int32_t m, const cox_refit_opts *opts, double *coef,
                     double *se, double *pval, double *loglik, int32_t *iters);

/* Negative log partial likelihood as a function of the linear predictor, for
 * automatic differentiation (the adjoint of the risk-set sums).
 * forward:  loss_b = -L(eta_b)   for eta dev [B][n] (float when eta_f64 = 0,
 *           double when 1); loss dev [B] double.  Keeps w and the reverse
 *           cumulative sums in the context for the next backward.
 * backward: grad_eta_b = -grad_loss_b * r_b, with r_b = delta - w_b * c_b the
 *           derivative of L at the eta of the last forward (Section 5.3's
 *           (I - P) delta).  grad_loss dev [B] double; grad_eta dev [B][n],
 *           float or double as in the forward.  The forward must have been
 *           called with the same B.  Neither call synchronises. */
cox_status cox_nll_forward(cox_ctx *ctx, const void *eta, int32_t eta_f64, int32_t B, double *loss);
cox_status cox_nll_backward(cox_ctx *ctx, const double *grad_loss, int32_t B, void *grad_eta);

/* Measurement: per-phase GPU time, taken with HIP events recorded on the
 * context's stream around each phase's launches (so it can run inside a timed
 * region).  Phases: COX_PHASE_XTR (the whole X~' r pass: residual quantisation
 * if any, the column sums, the fused proximal epilogue), COX_PHASE_RISK (the
 * risk-set kernels), COX_PHASE_ETA (the whole eta update or dense X~ beta
 * pass), COX_PHASE_XTR_KERNEL (each launch of the column-sum kernel alone:
 * the matrix-core X~' R kernel, or one vector X~' r launch per group of up to
 * 8 vectors), COX_PHASE_ETA_KERNEL (each launch of the matrix-core eta kernel
 * alone), COX_PHASE_COV (the covariate block's Z' r with its proximal step, and
 * its eta update; nothing without covariates), COX_PHASE_REFIT_HESSIAN (each
 * evaluation of the refit's information matrix), COX_PHASE_REFIT_SOLVE (each
 * Cholesky factorisation and Newton solve of the refit) and
 * COX_PHASE_PERSISTENT (each persistent launch of cox_fit_path, all its steps;
 * the other phases record nothing inside it).
 * cox_timing_enable(ctx, 1) starts recording and clears the totals; 0 stops.
 * cox_timing_read returns the summed milliseconds and the number of timed
 * launches of a phase since the last enable.  Synchronises. */
typedef enum {
    COX_PHASE_XTR = 0,
    COX_PHASE_RISK = 1,
    COX_PHASE_ETA = 2,
    COX_PHASE_XTR_KERNEL = 3,
    COX_PHASE_ETA_KERNEL = 4,
    COX_PHASE_COV = 5,
    COX_PHASE_REFIT_HESSIAN = 6,
    COX_PHASE_REFIT_SOLVE = 7,
    COX_PHASE_PERSISTENT = 8
} cox_phase;

/* The batched matrix-core passes (X~' R and the eta update, used when X holds
 * allele counts and B > 8) come in several pipeline shapes: COX_MFMA_VARIANTS
 * for X~' R, COX_MFMA_ETA_VARIANTS for the eta update.  The first batched call
 * times every shape on the live data (one untimed and three timed launches,
 * the median kept) and keeps the fastest (the
 * environment variable COXHIP_TUNE_CACHE names a file that caches the choice;
 * COXHIP_MFMA_VARIANT and COXHIP_ETA_VARIANT force one; COXHIP_ETA_SHARES sets
 * how many workgroups the eta shapes that share blocks between workgroups use,
 * at most the compute units, so that tests can make small problems share them).  This reports the
 * choices (-1: not yet tuned) and the tuning times in milliseconds (host
 * [COX_MFMA_VARIANTS] each, nullable; entries past a pass's shape count and
 * entries of a pass that was not timed are 0). */
#define COX_MFMA_VARIANTS 16
#define COX_MFMA_ETA_VARIANTS 13
cox_status cox_mfma_tuning(cox_ctx *ctx, int32_t *xtr_variant, int32_t *eta_variant, float *xtr_ms, float *eta_ms);
cox_status cox_timing_enable(cox_ctx *ctx, int32_t enable);
cox_status cox_timing_read(cox_ctx *ctx, int32_t phase, double *total_ms, int64_t *count);

/* Measurement: the columns of X the active-set eta updates of cox_fit_path
 * read since cox_timing_enable(ctx, 1) (the change list's length summed over
 * the steps; the multi-launch form with eta_mode 0 only -- dense passes and
 * persistent launches add nothing).  It gives the bytes of X a step moves
 * beside the full pass of X~' r.  eta_columns host [1].  Synchronises. */
cox_status cox_timing_columns(cox_ctx *ctx, int64_t *eta_columns);

/* Device memory the library holds at this moment, in bytes, over every live
 * context and the buffers of calls in progress (the static array of
 * cox_rank_path_noalloc is not counted: it belongs to the loaded library).
 * A failed call releases what it allocated, so the count returns to its
 * value before the call.  bytes host [1]. */
cox_status cox_device_bytes(int64_t *bytes);

#ifdef __cplusplus
}
#endif
#endif /* COX_H */
