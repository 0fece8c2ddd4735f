/*
 * cox_oracle.c -- plain double-precision CPU oracle for l1-regularised Cox
 * proportional-hazards regression by proximal gradient (ISTA).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code with the GPU path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product never does.
 *
 * What it follows (Ko, Zhou, Zhou and Won, "DistStat.jl", Section 5.3):
 *   - the Cox log partial likelihood L(beta) = sum_i delta_i [x_i'beta -
 *     log sum_{j: y_j >= y_i} exp(x_j'beta)]  (the displayed equation is read
 *     with the minus sign that its gradient requires);
 *   - the objective: maximise L(beta) - lambda ||beta||_1, here written as
 *     minimising f(beta) = -L(beta) + lambda ||beta||_1;
 *   - the iteration of Section 5.3: w_i = exp(x_i'beta), W_j = sum over the
 *     risk set {i: y_i >= y_j} of w_i, pi_ij = 1(y_i >= y_j) w_i / W_j,
 *     Delta = X'(I - P) delta, beta <- S(beta + sigma Delta);
 *   - the remark that, with the subjects sorted by non-increasing y, the
 *     risk-set sums are cumulative sums;
 *   - the soft-thresholding operator of Section 4.2 ("Dot syntax");
 *   - opnorm(., 2) by power iteration with tol 1e-6, maxiter 1000 (Section 4.3);
 *   - the lag-10 relative-objective stopping rule of Section 6;
 *   - Breslow's convention for tied times (Section 6);
 *   - Section 6's application, where sex and the top principal components
 *     enter the model unpenalised: a penalty factor pf_j >= 0 per column, the
 *     objective -L + lambda sum_j pf_j |beta_j| and the threshold
 *     sigma lambda pf_j (pf_j = 0: the column is unpenalised);
 *   - the unpenalised Cox fit on a chosen set of columns that the same section
 *     uses for its significance tests, here by Newton's method on L with its
 *     exact Hessian (the textbook maximiser; the paper names no method);
 *   - Section 6's ranking of the selected columns: by the largest lambda of
 *     the path at which a column's coefficient is nonzero, ties by the
 *     magnitude of the coefficient when it joins the model.
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - the ranking reads a path given in decreasing lambda, so a column's
 *     largest lambda is the first row where it is nonzero; columns tied on
 *     both the row and |coefficient| go in increasing column order;
 *   - the threshold of the prox is sigma*lambda (standard ISTA for the stated
 *     objective), not lambda;
 *   - risk sets use the observed times y, ties included (Breslow): tied
 *     subjects are all in each other's risk sets and tied events share W;
 *   - w is computed as exp(eta - max eta); every quantity that the iteration
 *     uses is invariant to this shift in exact arithmetic;
 *   - no normalisation of L by n or by the number of events;
 *   - with unpenalised columns U = {j : pf_j = 0}, lambda_max is the smallest
 *     lambda at which every penalised coefficient is zero at the optimum:
 *     max over penalised j of |g_j| / pf_j, with g the gradient of L at
 *     beta_U = the unpenalised maximiser over U and every other beta_j = 0.
 *
 * Parity status: every function here is pinned by the CPU tests (brute-force
 * risk sets, hand-derived closed forms, finite differences, a closed-form
 * minimiser, an independent quasi-Newton solver, an SVD, a finite-difference
 * Hessian).  None is unpinned.
 *
 * All arithmetic is IEEE double precision, evaluated in natural index order
 * except where OpenMP splits a loop over independent outputs.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_X_F64 0
#define ORACLE_X_F32 1
#define ORACLE_X_GENO 2 /* int8 allele counts, standardised as (g - mu_j) * s_j */

/* A dense n x p covariate matrix stored column by column: column j starts at
 * element j*ldx.  Values are read through xval(), always as doubles. */
typedef struct {
    int kind;
    const void *data;
    int64_t n, p, ldx;
    const double *mu; /* ORACLE_X_GENO only */
    const double *s;  /* ORACLE_X_GENO only */
} oracle_matrix;

static double xval(const oracle_matrix *X, int64_t i, int64_t j)
{
    int64_t at = j * X->ldx + i;
    switch (X->kind) {
    case ORACLE_X_F64: return ((const double *)X->data)[at];
    case ORACLE_X_F32: return (double)((const float *)X->data)[at];
    default: return ((double)((const int8_t *)X->data)[at] - X->mu[j]) * X->s[j];
    }
}

/* ------------------------------------------------------------------ order */

static const double *g_sort_time; /* qsort has no context argument */

static int by_time_desc(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    double ti = g_sort_time[i], tj = g_sort_time[j];
    if (ti > tj) return -1;
    if (ti < tj) return 1;
    return (i < j) ? -1 : (i > j); /* stable: keep index order within ties */
}

/* Subjects ordered by non-increasing observed time (Section 5.3), stable by
 * index.  order[k] is the subject at sorted position k.  For every position k,
 * gstart[k] and gend[k] are the first and last positions holding the same
 * time (its tie group).  Returns 0, or -1 on a non-finite time or no memory. */
int cox_oracle_order(int64_t n, const double *time, int64_t *order, int64_t *gstart, int64_t *gend)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(time[i])) return -1;
        order[i] = i;
    }
    g_sort_time = time;
    qsort(order, (size_t)n, sizeof(int64_t), by_time_desc);
    int64_t k = 0;
    while (k < n) {
        int64_t e = k;
        while (e + 1 < n && time[order[e + 1]] == time[order[k]]) ++e;
        for (int64_t q = k; q <= e; ++q) {
            gstart[q] = k;
            gend[q] = e;
        }
        k = e + 1;
    }
    return 0;
}

/* ------------------------------------------------------- partial likelihood */

/* Breslow log partial likelihood L at linear predictor eta, and its gradient
 * with respect to eta, r = (I - P) delta (Section 5.3):
 *   m     = max_i eta_i
 *   w_i   = exp(eta_i - m)
 *   W_i   = sum_{j: y_j >= y_i} w_j     (a cumulative sum in sorted order,
 *                                        read at the end of i's tie group)
 *   L     = sum_i delta_i (eta_i - m - log W_i)
 *   (P delta)_k = sum_i pi_ki delta_i = w_k sum_{i: y_i <= y_k} delta_i / W_i
 *                                       (a reverse cumulative sum, read at the
 *                                        start of k's tie group)
 *   r_k   = delta_k - (P delta)_k
 * r is written in original subject order.  Returns L. */
static double loglik_resid_sorted(int64_t n, const double *eta, const int32_t *event,
                                  const int64_t *order, const int64_t *gstart, const int64_t *gend,
                                  double *r, double *work /* 3n */)
{
    double *w = work, *S = work + n, *T = work + 2 * n;
    double m = -INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (eta[i] > m) m = eta[i];
    if (n == 0) return 0.0;

    double acc = 0.0;
    for (int64_t k = 0; k < n; ++k) { /* cumulative sum in decreasing time */
        w[k] = exp(eta[order[k]] - m);
        acc += w[k];
        S[k] = acc;
    }
    double L = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        int64_t i = order[k];
        if (event[i]) L += eta[i] - m - log(S[gend[k]]);
    }
    acc = 0.0;
    for (int64_t k = n - 1; k >= 0; --k) { /* reverse cumulative sum of delta/W */
        int64_t i = order[k];
        if (event[i]) acc += 1.0 / S[gend[k]];
        T[k] = acc;
    }
    if (r)
        for (int64_t k = 0; k < n; ++k) {
            int64_t i = order[k];
            r[i] = (double)(event[i] != 0) - w[k] * T[gstart[k]];
        }
    return L;
}

/* Public form: sorts internally.  r (length n) may be NULL.  Returns 0 or -1. */
int cox_oracle_loglik(int64_t n, const double *eta, const double *time, const int32_t *event,
                      double *L_out, double *r)
{
    int64_t *order = malloc(sizeof(int64_t) * (size_t)(3 * n + 1));
    double *work = malloc(sizeof(double) * (size_t)(3 * n + 1));
    if (!order || !work) { free(order); free(work); return -1; }
    int64_t *gstart = order + n, *gend = order + 2 * n;
    if (cox_oracle_order(n, time, order, gstart, gend)) { free(order); free(work); return -1; }
    *L_out = loglik_resid_sorted(n, eta, event, order, gstart, gend, r, work);
    free(order);
    free(work);
    return 0;
}

/* ---------------------------------------------------------- linear algebra */

/* eta = X beta.  OpenMP splits the rows into blocks of 256; within a block the
 * columns are visited in order, so each eta_i is summed over j = 0, 1, ...
 * (terms with beta_j = 0 are skipped: they add exactly zero). */
static void xbeta(const oracle_matrix *X, const double *beta, double *eta)
{
    int64_t n = X->n, p = X->p;
#pragma omp parallel for schedule(static)
    for (int64_t b0 = 0; b0 < n; b0 += 256) {
        int64_t b1 = (b0 + 256 < n) ? b0 + 256 : n;
        for (int64_t i = b0; i < b1; ++i) eta[i] = 0.0;
        for (int64_t j = 0; j < p; ++j) {
            if (beta[j] == 0.0) continue;
            for (int64_t i = b0; i < b1; ++i) eta[i] += xval(X, i, j) * beta[j];
        }
    }
}

/* g = X' r.  OpenMP splits the columns; each column's sum runs over i in order. */
static void xtr(const oracle_matrix *X, const double *r, double *g)
{
    int64_t n = X->n, p = X->p;
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < p; ++j) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += xval(X, i, j) * r[i];
        g[j] = s;
    }
}

static int make_matrix(oracle_matrix *X, int kind, const void *data, int64_t n, int64_t p, int64_t ldx,
                       const double *mu, const double *s)
{
    if (n < 0 || p < 0 || ldx < n || !data) return -1;
    if (kind == ORACLE_X_GENO && (!mu || !s)) return -1;
    if (kind != ORACLE_X_F64 && kind != ORACLE_X_F32 && kind != ORACLE_X_GENO) return -1;
    X->kind = kind; X->data = data; X->n = n; X->p = p; X->ldx = ldx; X->mu = mu; X->s = s;
    return 0;
}

int cox_oracle_xbeta(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                     const double *s, const double *beta, double *eta)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s)) return -1;
    xbeta(&X, beta, eta);
    return 0;
}

int cox_oracle_xtr(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                   const double *s, const double *r, double *g)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s)) return -1;
    xtr(&X, r, g);
    return 0;
}

/* Soft-thresholding operator S_t(x) (Section 4.2): x - t above t, x + t below
 * -t, zero in between. */
double cox_oracle_soft_threshold(double x, double t)
{
    if (x > t) return x - t;
    if (x < -t) return x + t;
    return 0.0;
}

/* ------------------------------------------------------------ loss, grad */

/* Negative log partial likelihood -L(beta) and, if g is not NULL, the
 * gradient of L, g = X'(I - P) delta (Section 5.3, "Delta").  Returns 0/-1. */
int cox_oracle_loss_grad(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                         const double *s, const double *time, const int32_t *event, const double *beta,
                         double *negL, double *g)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s)) return -1;
    double *eta = malloc(sizeof(double) * (size_t)(n + 1));
    double *r = malloc(sizeof(double) * (size_t)(n + 1));
    if (!eta || !r) { free(eta); free(r); return -1; }
    xbeta(&X, beta, eta);
    double L;
    if (cox_oracle_loglik(n, eta, time, event, &L, r)) { free(eta); free(r); return -1; }
    *negL = -L;
    if (g) xtr(&X, r, g);
    free(eta);
    free(r);
    return 0;
}

/* lambda_max = max_j |g_j(0)|: the smallest lambda at which beta = 0 is a
 * fixed point of the iteration (for any step size). */
int cox_oracle_lambda_max(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                          const double *s, const double *time, const int32_t *event, double *lambda_max)
{
    double *beta = calloc((size_t)(p + 1), sizeof(double));
    double *g = malloc(sizeof(double) * (size_t)(p + 1));
    if (!beta || !g) { free(beta); free(g); return -1; }
    double negL;
    int rc = cox_oracle_loss_grad(kind, data, n, p, ldx, mu, s, time, event, beta, &negL, g);
    double mx = 0.0;
    for (int64_t j = 0; rc == 0 && j < p; ++j)
        if (fabs(g[j]) > mx) mx = fabs(g[j]);
    *lambda_max = mx;
    free(beta);
    free(g);
    return rc;
}

/* --------------------------------------------------------- power iteration */

/* SplitMix64 (Steele, Lea and Flood, 2014): x advances by the golden-ratio
 * increment, then is mixed by two xor-shift-multiply rounds. */
static uint64_t splitmix64_next(uint64_t *state)
{
    uint64_t z = (*state += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* ||X||_2^2 by power iteration on X'X (Section 4.3, opnorm(a, 2; method =
 * "power")).  The start vector has entries uniform on [-1, 1) drawn from
 * SplitMix64 seeded with `seed` (top 53 bits of each output).  Each step:
 * u = X v; v' = X'u; estimate = ||X v||^2 for the unit vector v; v = v'/||v'||.
 * Stops when the estimate changes by less than tol relative to itself, or
 * after maxiter steps.  Returns 0/-1; *iters_out gets the steps taken. */
int cox_oracle_opnorm2(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                       const double *s, double tol, int32_t maxiter, uint64_t seed, double *s2_out,
                       int32_t *iters_out)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s) || p < 1 || n < 1) return -1;
    double *v = malloc(sizeof(double) * (size_t)p), *g = malloc(sizeof(double) * (size_t)p);
    double *u = malloc(sizeof(double) * (size_t)n);
    if (!v || !g || !u) { free(v); free(g); free(u); return -1; }
    uint64_t st = seed;
    double nv = 0.0;
    for (int64_t j = 0; j < p; ++j) {
        v[j] = (double)(splitmix64_next(&st) >> 11) * 0x1.0p-52 - 1.0;
        nv += v[j] * v[j];
    }
    nv = sqrt(nv);
    for (int64_t j = 0; j < p; ++j) v[j] /= nv;
    double est = 0.0;
    int32_t it = 0;
    while (it < maxiter) {
        xbeta(&X, v, u);
        double nu = 0.0;
        for (int64_t i = 0; i < n; ++i) nu += u[i] * u[i];
        xtr(&X, u, g);
        double ng = 0.0;
        for (int64_t j = 0; j < p; ++j) ng += g[j] * g[j];
        ng = sqrt(ng);
        ++it;
        double prev = est;
        est = nu;
        if (ng == 0.0) break;
        for (int64_t j = 0; j < p; ++j) v[j] = g[j] / ng;
        if (it > 1 && fabs(est - prev) < tol * est) break;
    }
    *s2_out = est;
    if (iters_out) *iters_out = it;
    free(v); free(g); free(u);
    return 0;
}

/* ------------------------------------------------------------------- ISTA */

/* Proximal gradient (ISTA) for min f(beta) = -L(beta) + lambda sum_j pf_j
 * |beta_j| (Section 5.3; pf = NULL means pf_j = 1 for every j, the plain l1
 * penalty), from the start point in beta[] (in/out).
 *
 * At iterate k (k = 0, 1, ...): eta = X beta_k; the risk-set sums give L and
 * r; f_k = -L + lambda sum_j pf_j |beta_kj| is recorded in obj_trace[k] (if
 * given); then
 *   - if k >= lag and |f_k - f_{k-lag}| / (|f_k| + 1) < tol, stop (Section 6's
 *     rule) with beta_k;
 *   - if k == max_iter, stop with beta_k;
 *   - otherwise beta_{k+1,j} = S_{sigma lambda pf_j}(beta_kj + sigma (X'r)_j).
 * *iters_out = k at the stop (the number of steps taken).  Returns 0 when the
 * rule fired, 1 when max_iter was reached, -1 on bad input or no memory, -2
 * when the objective became non-finite. */
static int fit_impl(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                    const double *s, const double *time, const int32_t *event, double lambda, const double *pf,
                    double sigma, int32_t max_iter, double tol, int32_t lag, double *beta, double *obj_trace,
                    double *beta_hist, int32_t *iters_out)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s) || lag < 1 || max_iter < 0) return -1;
    for (int64_t j = 0; pf && j < p; ++j)
        if (!(pf[j] >= 0.0) || !isfinite(pf[j])) return -1;
    int64_t *order = malloc(sizeof(int64_t) * (size_t)(3 * n + 1));
    double *work = malloc(sizeof(double) * (size_t)(3 * n + 1));
    double *eta = malloc(sizeof(double) * (size_t)(n + 1));
    double *r = malloc(sizeof(double) * (size_t)(n + 1));
    double *g = malloc(sizeof(double) * (size_t)(p + 1));
    double *hist = malloc(sizeof(double) * (size_t)(max_iter + 1));
    int rc = -1;
    if (!order || !work || !eta || !r || !g || !hist) goto out;
    int64_t *gstart = order + n, *gend = order + 2 * n;
    if (cox_oracle_order(n, time, order, gstart, gend)) goto out;

    for (int32_t k = 0;; ++k) {
        xbeta(&X, beta, eta);
        double L = loglik_resid_sorted(n, eta, event, order, gstart, gend, r, work);
        double l1 = 0.0;
        for (int64_t j = 0; j < p; ++j) l1 += (pf ? pf[j] : 1.0) * fabs(beta[j]);
        double f = -L + lambda * l1;
        hist[k] = f;
        if (obj_trace) obj_trace[k] = f;
        if (beta_hist) memcpy(beta_hist + (size_t)k * (size_t)p, beta, sizeof(double) * (size_t)p);
        if (!isfinite(f)) { rc = -2; *iters_out = k; break; }
        if (k >= lag && fabs(f - hist[k - lag]) / (fabs(f) + 1.0) < tol) { rc = 0; *iters_out = k; break; }
        if (k == max_iter) { rc = 1; *iters_out = k; break; }
        xtr(&X, r, g);
        for (int64_t j = 0; j < p; ++j)
            beta[j] = cox_oracle_soft_threshold(beta[j] + sigma * g[j], sigma * lambda * (pf ? pf[j] : 1.0));
    }
out:
    free(order); free(work); free(eta); free(r); free(g); free(hist);
    return rc;
}

int cox_oracle_fit_pf(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                      const double *s, const double *time, const int32_t *event, double lambda,
                      const double *pf, double sigma, int32_t max_iter, double tol, int32_t lag, double *beta,
                      double *obj_trace, int32_t *iters_out)
{
    return fit_impl(kind, data, n, p, ldx, mu, s, time, event, lambda, pf, sigma, max_iter, tol, lag, beta,
                    obj_trace, NULL, iters_out);
}

/* The same iteration with every pf_j = 1, also recording each iterate:
 * beta_hist[k*p + j] = beta_kj for k = 0 .. the step at which it stops
 * (beta_hist holds max_iter + 1 rows of p). */
int cox_oracle_fit_hist(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                        const double *s, const double *time, const int32_t *event, double lambda, double sigma,
                        int32_t max_iter, double tol, int32_t lag, double *beta, double *obj_trace,
                        double *beta_hist, int32_t *iters_out)
{
    if (!beta_hist) return -1;
    return fit_impl(kind, data, n, p, ldx, mu, s, time, event, lambda, NULL, sigma, max_iter, tol, lag, beta,
                    obj_trace, beta_hist, iters_out);
}

/* The plain l1 problem: cox_oracle_fit_pf with every pf_j = 1. */
int cox_oracle_fit(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                   const double *s, const double *time, const int32_t *event, double lambda, double sigma,
                   int32_t max_iter, double tol, int32_t lag, double *beta, double *obj_trace,
                   int32_t *iters_out)
{
    return cox_oracle_fit_pf(kind, data, n, p, ldx, mu, s, time, event, lambda, NULL, sigma, max_iter, tol, lag,
                             beta, obj_trace, iters_out);
}

/* ------------------------------------------------- unpenalised Newton fit */

/* Gradient and Hessian of L with respect to the coefficients of the m columns
 * cols[0..m-1], at linear predictor eta (Breslow ties).  With the risk set
 * R_i = {j : y_j >= y_i}, w_j = exp(eta_j - max eta), and for each event i
 *   W_i   = sum_{j in R_i} w_j,
 *   S1_i  = sum_{j in R_i} w_j x_j          (m-vector over the chosen columns),
 *   S2_i  = sum_{j in R_i} w_j x_j x_j'     (m x m),
 * L's gradient is sum_i delta_i (x_i - S1_i / W_i) and its Hessian is
 * -sum_i delta_i (S2_i / W_i - S1_i S1_i' / W_i^2).  In sorted order the sums
 * over R_i are running sums, complete at the end of i's tie group: a tie
 * group is accumulated whole, then its events are added.  grad [m], hess
 * [m*m] row-major.  Returns L. */
static double loglik_grad_hess(const oracle_matrix *X, const int64_t *cols, int64_t m, const double *eta,
                               const int32_t *event, const int64_t *order, const int64_t *gend, double *grad,
                               double *hess, double *S1 /* m */, double *S2 /* m*m */, double *xk /* m */)
{
    const int64_t n = X->n;
    double mx = -INFINITY;
    for (int64_t i = 0; i < n; ++i)
        if (eta[i] > mx) mx = eta[i];
    double W = 0.0, L = 0.0;
    for (int64_t a = 0; a < m; ++a) S1[a] = grad[a] = 0.0;
    for (int64_t a = 0; a < m * m; ++a) S2[a] = hess[a] = 0.0;
    int64_t k = 0;
    while (k < n) {
        const int64_t e = gend[k];
        for (int64_t q = k; q <= e; ++q) { /* the tie group joins the running sums */
            const int64_t i = order[q];
            const double w = exp(eta[i] - mx);
            for (int64_t a = 0; a < m; ++a) xk[a] = xval(X, i, cols[a]);
            W += w;
            for (int64_t a = 0; a < m; ++a) {
                S1[a] += w * xk[a];
                for (int64_t b = 0; b < m; ++b) S2[a * m + b] += w * xk[a] * xk[b];
            }
        }
        for (int64_t q = k; q <= e; ++q) { /* its events see the whole risk set */
            const int64_t i = order[q];
            if (!event[i]) continue;
            L += eta[i] - mx - log(W);
            for (int64_t a = 0; a < m; ++a) {
                grad[a] += xval(X, i, cols[a]) - S1[a] / W;
                for (int64_t b = 0; b < m; ++b) hess[a * m + b] -= S2[a * m + b] / W - S1[a] * S1[b] / (W * W);
            }
        }
        k = e + 1;
    }
    return L;
}

/* Solve A x = b for a symmetric positive definite m x m matrix A (row-major) by
 * Cholesky factorisation; A is overwritten by its factor.  Returns 0, or -1 when
 * A is not numerically positive definite. */
static int cholesky_factor(double *A, int64_t m)
{
    for (int64_t j = 0; j < m; ++j) {
        double d = A[j * m + j];
        for (int64_t k = 0; k < j; ++k) d -= A[j * m + k] * A[j * m + k];
        if (!(d > 0.0)) return -1;
        d = sqrt(d);
        A[j * m + j] = d;
        for (int64_t i = j + 1; i < m; ++i) {
            double v = A[i * m + j];
            for (int64_t k = 0; k < j; ++k) v -= A[i * m + k] * A[j * m + k];
            A[i * m + j] = v / d;
        }
    }
    return 0;
}

/* x <- (L L')^{-1} x with the factor from cholesky_factor */
static void cholesky_subst(const double *A, int64_t m, double *x)
{
    for (int64_t i = 0; i < m; ++i) { /* forward: L y = b */
        double v = x[i];
        for (int64_t k = 0; k < i; ++k) v -= A[i * m + k] * x[k];
        x[i] = v / A[i * m + i];
    }
    for (int64_t i = m - 1; i >= 0; --i) { /* back: L' x = y */
        double v = x[i];
        for (int64_t k = i + 1; k < m; ++k) v -= A[k * m + i] * x[k];
        x[i] = v / A[i * m + i];
    }
}

static int cholesky_solve(double *A, int64_t m, double *x)
{
    if (cholesky_factor(A, m)) return -1;
    cholesky_subst(A, m, x);
    return 0;
}

/* Unpenalised maximum partial likelihood over the m columns cols[] with every
 * other coefficient fixed at beta_fixed (NULL: zero), by Newton's method with
 * step halving: from beta_sub (in/out, length m), each step solves
 * (-H) d = g and takes the largest of d, d/2, d/4, ... that does not lower L;
 * it stops when max_a |g_a| <= gtol (after the step), or after maxit steps.
 * On return, if cov is not NULL it holds the inverse of -H at the result
 * (m x m, row-major: the estimated covariance of beta_sub, whose diagonal gives
 * the standard errors of Wald tests).  *iters_out = Newton steps taken.
 * Returns 0 when converged, 1 at maxit, -1 on bad input or no memory, -2 when
 * -H is not positive definite. */
int cox_oracle_newton(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                      const double *s, const double *time, const int32_t *event, const int64_t *cols, int64_t m,
                      const double *beta_fixed, double *beta_sub, int32_t maxit, double gtol, double *cov,
                      int32_t *iters_out)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s) || m < 1 || m > 1024 || maxit < 0 || n < 1) return -1;
    for (int64_t a = 0; a < m; ++a)
        if (cols[a] < 0 || cols[a] >= p) return -1;
    int64_t *order = malloc(sizeof(int64_t) * (size_t)(3 * n));
    double *beta = malloc(sizeof(double) * (size_t)p);
    double *eta = malloc(sizeof(double) * (size_t)n);
    double *grad = malloc(sizeof(double) * (size_t)m), *hess = malloc(sizeof(double) * (size_t)(m * m));
    double *fac = malloc(sizeof(double) * (size_t)(m * m)), *d = malloc(sizeof(double) * (size_t)m);
    double *S1 = malloc(sizeof(double) * (size_t)m), *S2 = malloc(sizeof(double) * (size_t)(m * m));
    double *xk = malloc(sizeof(double) * (size_t)m), *trial = malloc(sizeof(double) * (size_t)m);
    int rc = -1;
    int32_t it = 0;
    if (!order || !beta || !eta || !grad || !hess || !fac || !d || !S1 || !S2 || !xk || !trial) goto out;
    int64_t *gstart = order + n, *gend = order + 2 * n;
    if (cox_oracle_order(n, time, order, gstart, gend)) goto out;
    for (int64_t j = 0; j < p; ++j) beta[j] = beta_fixed ? beta_fixed[j] : 0.0;
    for (int64_t a = 0; a < m; ++a) beta[cols[a]] = beta_sub[a];
    xbeta(&X, beta, eta);
    double L = loglik_grad_hess(&X, cols, m, eta, event, order, gend, grad, hess, S1, S2, xk);
    rc = 1;
    for (;;) {
        double gmax = 0.0;
        for (int64_t a = 0; a < m; ++a)
            if (fabs(grad[a]) > gmax) gmax = fabs(grad[a]);
        if (gmax <= gtol) { rc = 0; break; }
        if (it >= maxit) { rc = 1; break; }
        for (int64_t a = 0; a < m * m; ++a) fac[a] = -hess[a];
        memcpy(d, grad, sizeof(double) * (size_t)m);
        if (cholesky_solve(fac, m, d)) { rc = -2; break; }
        /* predicted gain of the full step, g'd; once it is at the rounding level
         * of L the full step is taken unchecked (the quadratic model is exact
         * to that order there), else the step is halved until L does not fall */
        double gain = 0.0;
        for (int64_t a = 0; a < m; ++a) gain += grad[a] * d[a];
        const int pure = gain <= 1e-12 * (1.0 + fabs(L));
        double t = 1.0, Lt = -INFINITY;
        for (int half = 0; half < 60; ++half, t *= 0.5) {
            for (int64_t a = 0; a < m; ++a) {
                trial[a] = beta_sub[a] + t * d[a];
                beta[cols[a]] = trial[a];
            }
            xbeta(&X, beta, eta);
            Lt = loglik_grad_hess(&X, cols, m, eta, event, order, gend, grad, hess, S1, S2, xk);
            if (Lt >= L || pure) break;
        }
        ++it;
        if (pure && isfinite(Lt)) {
            memcpy(beta_sub, trial, sizeof(double) * (size_t)m);
            L = Lt;
            continue;
        }
        if (!(Lt >= L)) { /* no ascent along the Newton direction (rounding level): stay at beta_sub */
            for (int64_t a = 0; a < m; ++a) beta[cols[a]] = beta_sub[a];
            xbeta(&X, beta, eta);
            loglik_grad_hess(&X, cols, m, eta, event, order, gend, grad, hess, S1, S2, xk);
            rc = 1;
            break;
        }
        memcpy(beta_sub, trial, sizeof(double) * (size_t)m);
        L = Lt;
    }
    if (cov && rc >= 0) {
        /* inverse of -H, column by column from one factorisation */
        for (int64_t a = 0; a < m * m; ++a) fac[a] = -hess[a];
        if (cholesky_factor(fac, m)) {
            rc = -2;
        } else {
            for (int64_t b = 0; b < m; ++b) {
                for (int64_t a = 0; a < m; ++a) d[a] = (a == b) ? 1.0 : 0.0;
                cholesky_subst(fac, m, d);
                for (int64_t a = 0; a < m; ++a) cov[a * m + b] = d[a];
            }
        }
    }
out:
    if (iters_out) *iters_out = it;
    free(order); free(beta); free(eta); free(grad); free(hess); free(fac); free(d); free(S1); free(S2);
    free(xk); free(trial);
    return rc;
}

/* lambda_max with penalty factors: with U = {j : pf_j = 0} (pf = NULL: none),
 * beta_U = the unpenalised maximiser over U (Newton, gradient below gtol) and
 * every other coefficient zero, the largest |g_j| / pf_j over penalised j of
 * the gradient g of L there.  beta_u_out (nullable) receives beta_U in
 * increasing column order.  Returns 0, -1 on bad input, -2 when the Newton
 * fit fails. */
int cox_oracle_lambda_max_pf(int kind, const void *data, int64_t n, int64_t p, int64_t ldx, const double *mu,
                             const double *s, const double *time, const int32_t *event, const double *pf,
                             double gtol, double *lambda_max, double *beta_u_out)
{
    oracle_matrix X;
    if (make_matrix(&X, kind, data, n, p, ldx, mu, s)) return -1;
    int64_t m = 0;
    int64_t *cols = malloc(sizeof(int64_t) * (size_t)(p + 1));
    double *beta = calloc((size_t)(p + 1), sizeof(double));
    double *bu = calloc((size_t)(p + 1), sizeof(double));
    double *g = malloc(sizeof(double) * (size_t)(p + 1));
    int rc = -1;
    if (!cols || !beta || !bu || !g) goto out;
    for (int64_t j = 0; j < p; ++j) {
        if (pf && (!(pf[j] >= 0.0) || !isfinite(pf[j]))) goto out;
        if (pf && pf[j] == 0.0) cols[m++] = j;
    }
    if (m > 0) {
        int32_t it;
        int nr = cox_oracle_newton(kind, data, n, p, ldx, mu, s, time, event, cols, m, NULL, bu, 200, gtol, NULL,
                                   &it);
        if (nr != 0) { rc = -2; goto out; }
        for (int64_t a = 0; a < m; ++a) beta[cols[a]] = bu[a];
    }
    double negL;
    rc = cox_oracle_loss_grad(kind, data, n, p, ldx, mu, s, time, event, beta, &negL, g);
    double mx = 0.0;
    for (int64_t j = 0; rc == 0 && j < p; ++j) {
        const double f = pf ? pf[j] : 1.0;
        if (f > 0.0 && fabs(g[j]) / f > mx) mx = fabs(g[j]) / f;
    }
    *lambda_max = mx;
    if (beta_u_out) memcpy(beta_u_out, bu, sizeof(double) * (size_t)m);
out:
    free(cols); free(beta); free(bu); free(g);
    return rc;
}

/* Section 6's ranking of a lambda path.  path is L x p (row l: the
 * coefficients at the l-th lambda, the lambdas decreasing; row stride ldp).
 * entry[j] = the first row where column j is nonzero (-1: never), coef[j] =
 * |path[entry[j]][j]| (0 if never), order[0..m) = the columns with entry >= 0
 * by entry ascending, then coef descending, then column ascending; m is
 * returned through m_out.  Returns 0, or -1 on bad input. */
static const int32_t *rank_entry;
static const float *rank_coef;

static int rank_cmp(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    if (rank_entry[x] != rank_entry[y]) return rank_entry[x] < rank_entry[y] ? -1 : 1;
    if (rank_coef[x] != rank_coef[y]) return rank_coef[x] > rank_coef[y] ? -1 : 1;
    return x < y ? -1 : (x > y);
}

int cox_oracle_rank_path(const float *path, int32_t L, int64_t p, int64_t ldp, int32_t *entry, float *coef,
                         int64_t *order, int64_t *m_out)
{
    if (!path || L < 1 || p < 1 || ldp < p || !entry || !coef || !order || !m_out) return -1;
    int64_t m = 0;
    for (int64_t j = 0; j < p; ++j) {
        entry[j] = -1;
        coef[j] = 0.0f;
        for (int32_t l = 0; l < L; ++l) {
            const float v = path[(int64_t)l * ldp + j];
            if (v != 0.0f) {
                entry[j] = l;
                coef[j] = fabsf(v);
                break;
            }
        }
        if (entry[j] >= 0) order[m++] = j;
    }
    rank_entry = entry;
    rank_coef = coef;
    qsort(order, (size_t)m, sizeof(int64_t), rank_cmp);
    *m_out = m;
    return 0;
}
