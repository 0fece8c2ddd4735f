/*
 * nmf_oracle.c -- plain double-precision CPU oracle for nonnegative matrix
 * factorisation, X ~ V W with V >= 0 (m x r) and W >= 0 (r x n), the cost
 * f(V, W) = ||X - V W||_F^2 (Section 5.1).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU library is checked against.  It shares no code with the GPU path.  Only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it; the product never does.
 *
 * What it follows (Ko, Zhou, Zhou and Won, "DistStat.jl", Section 5.1):
 *   - the multiplicative updates of Lee and Seung:
 *       V <- V .* (X W') ./ (V W W' + eps),   then, with that new V,
 *       W <- W .* (V' X) ./ (V' V W + eps);
 *   - the alternating projected gradient updates of Lin:
 *       V <- max(0, V - sigma (V W W' - X W')),  sigma = 1 / (2 ||W W'||_F^2 + eps),
 *       then, with that new V,
 *       W <- max(0, W - tau (V' V W - V' X)),    tau = 1 / (2 ||V' V||_F^2 + eps);
 *   - eps is added to each denominator, as in the paper's loop.
 *
 * Readings taken where the paper is silent or inconsistent:
 *   - the displayed multiplicative W update writes V' V' W in its
 *     denominator; V' V W (the gradient's term, and the paper's loop) is used;
 *   - the step sizes of the displayed APG formulas carry no eps, the loop adds
 *     eps to the denominator; the loop's form is used.
 *
 * The factors are stored as the paper's loop stores them: Vt = V' (r x m) and W
 * (r x n), both row-major; X is m x n row-major (row i at X + i*ldx).
 *
 * Parity status: pinned by the CPU tests (monotone decrease of both updates,
 * the fixed point of an exact factorisation under the multiplicative update,
 * the KKT conditions at convergence, exact recovery of a low-rank X, and the
 * objective identity against a direct evaluation).  None is unpinned.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* f = ||X - V W||_F^2 = sum_ij (X_ij - sum_a Vt[a][i] W[a][j])^2, directly. */
double nmf_oracle_objective(const float *X, int64_t m, int64_t n, int64_t ldx, int32_t r, const double *Vt,
                            const double *W)
{
    double f = 0.0;
#pragma omp parallel for reduction(+ : f) schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double v = 0.0;
            for (int32_t a = 0; a < r; ++a) v += Vt[a * m + i] * W[a * n + j];
            const double d = (double)X[i * ldx + j] - v;
            f += d * d;
        }
    }
    return f;
}

/* One iteration (V update, then W update) of algorithm algo (0: multiplicative,
 * 1: APG), in place.  Returns 0, or -1 on bad input or no memory. */
int nmf_oracle_step(const float *X, int64_t m, int64_t n, int64_t ldx, int32_t r, int32_t algo, double eps,
                    double *Vt, double *W)
{
    if (m < 1 || n < 1 || ldx < n || r < 1 || (algo != 0 && algo != 1)) return -1;
    double *WXt = malloc(sizeof(double) * (size_t)(r * m)); /* W X' : r x m */
    double *WWt = malloc(sizeof(double) * (size_t)(r * r));
    double *VtX = malloc(sizeof(double) * (size_t)(r * n)); /* V' X : r x n */
    double *VtV = malloc(sizeof(double) * (size_t)(r * r));
    if (!WXt || !WWt || !VtX || !VtV) {
        free(WXt); free(WWt); free(VtX); free(VtV);
        return -1;
    }
    /* ---- V update */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i)
        for (int32_t a = 0; a < r; ++a) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += W[a * n + j] * (double)X[i * ldx + j];
            WXt[a * m + i] = s;
        }
    for (int32_t a = 0; a < r; ++a)
        for (int32_t b = 0; b < r; ++b) {
            double s = 0.0;
            for (int64_t j = 0; j < n; ++j) s += W[a * n + j] * W[b * n + j];
            WWt[a * r + b] = s;
        }
    double sigma = 0.0;
    if (algo == 1) {
        double s = 0.0;
        for (int32_t q = 0; q < r * r; ++q) s += WWt[q] * WWt[q];
        sigma = 1.0 / (2.0 * s + eps);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double old[256];
        for (int32_t a = 0; a < r; ++a) old[a] = Vt[a * m + i];
        for (int32_t a = 0; a < r; ++a) {
            double den = 0.0; /* (W W' V')[a][i] */
            for (int32_t b = 0; b < r; ++b) den += WWt[a * r + b] * old[b];
            if (algo == 0)
                Vt[a * m + i] = old[a] * WXt[a * m + i] / (den + eps);
            else
                Vt[a * m + i] = fmax(0.0, old[a] - sigma * (den - WXt[a * m + i]));
        }
    }
    /* ---- W update with the new V */
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j)
        for (int32_t a = 0; a < r; ++a) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += Vt[a * m + i] * (double)X[i * ldx + j];
            VtX[a * n + j] = s;
        }
    for (int32_t a = 0; a < r; ++a)
        for (int32_t b = 0; b < r; ++b) {
            double s = 0.0;
            for (int64_t i = 0; i < m; ++i) s += Vt[a * m + i] * Vt[b * m + i];
            VtV[a * r + b] = s;
        }
    double tau = 0.0;
    if (algo == 1) {
        double s = 0.0;
        for (int32_t q = 0; q < r * r; ++q) s += VtV[q] * VtV[q];
        tau = 1.0 / (2.0 * s + eps);
    }
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < n; ++j) {
        double old[256];
        for (int32_t a = 0; a < r; ++a) old[a] = W[a * n + j];
        for (int32_t a = 0; a < r; ++a) {
            double den = 0.0; /* (V' V W)[a][j] */
            for (int32_t b = 0; b < r; ++b) den += VtV[a * r + b] * old[b];
            if (algo == 0)
                W[a * n + j] = old[a] * VtX[a * n + j] / (den + eps);
            else
                W[a * n + j] = fmax(0.0, old[a] - tau * (den - VtX[a * n + j]));
        }
    }
    free(WXt); free(WWt); free(VtX); free(VtV);
    return 0;
}

/* iters iterations; obj_trace (nullable, [iters + 1]) receives f before the
 * first and after each iteration.  r <= 256.  Returns 0 or -1. */
int nmf_oracle_run(const float *X, int64_t m, int64_t n, int64_t ldx, int32_t r, int32_t algo, double eps,
                   int32_t iters, double *Vt, double *W, double *obj_trace)
{
    if (r < 1 || r > 256 || iters < 0) return -1;
    if (obj_trace) obj_trace[0] = nmf_oracle_objective(X, m, n, ldx, r, Vt, W);
    for (int32_t k = 0; k < iters; ++k) {
        if (nmf_oracle_step(X, m, n, ldx, r, algo, eps, Vt, W)) return -1;
        if (obj_trace) obj_trace[k + 1] = nmf_oracle_objective(X, m, n, ldx, r, Vt, W);
    }
    return 0;
}
