/*
 * nmf.h -- C ABI of the nonnegative matrix factorisation in libcoxhip, the
 * paper's other GPU workload (Ko, Zhou, Zhou and Won, "DistStat.jl",
 * Section 5.1): X ~ V W with X (m x n) nonnegative, V (m x r) and W (r x n)
 * nonnegative, minimising f(V, W) = ||X - V W||_F^2.
 *
 * Data layout.  X is FP32, row-major, row i at X + i*ldx (ldx >= n), device
 * memory, BORROWED (valid and unchanged while the context exists).  The
 * factors are held as the paper's loop holds them, V' (r x m) and W (r x n),
 * row-major, in FP64 device memory owned by the caller.  Every product with X
 * is formed and summed in FP64.
 *
 * Status codes, error behaviour and stream ordering are those of cox.h: every
 * call returns a cox_status, argument errors are reported before any device
 * work, and all work runs on the stream given to nmf_setup.
 */
#ifndef NMF_H
#define NMF_H

#include <stddef.h>
#include <stdint.h>

#include "cox.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_ctx nmf_ctx;

#define NMF_MAX_RANK 64

typedef enum {
    NMF_MULTIPLICATIVE = 0, /* Lee and Seung: V <- V .* (X W') ./ (V W W' + eps), then
                               W <- W .* (V' X) ./ (V' V W + eps) with the new V */
    NMF_APG = 1             /* alternating projected gradient (Lin):
                               V <- max(0, V - sigma (V W W' - X W')), sigma = 1/(2||W W'||_F^2 + eps), then
                               W <- max(0, W - tau (V' V W - V' X)),   tau = 1/(2||V' V||_F^2 + eps) */
} nmf_algo;

/* Create a context for X (m x n, 1 <= m, n < 2^31, ldx >= n) and rank r
 * (1..NMF_MAX_RANK): allocates the split partials and computes ||X||_F^2 once.
 * INVALID_ARG, OUT_OF_MEMORY or DEVICE with *out NULL on failure.
 * Synchronises. */
cox_status nmf_setup(nmf_ctx **out, const float *X, int64_t m, int64_t n, int64_t ldx, int32_t r,
                     void *hip_stream);
cox_status nmf_destroy(nmf_ctx *ctx);
cox_status nmf_last_error(const nmf_ctx *ctx, char *buf, size_t len);

/* iters iterations of algo (nmf_algo) from the given factors, in place, in the
 * order of Section 5.1's loop (the V update, then the W update with the new V):
 *   Vt  dev [r][m] double, in/out;  W dev [r][n] double, in/out
 *   eps >= 0 added to the denominators (the paper's loop uses 1e-10)
 *   obj host [1] or NULL: f(V, W) at the end, from ||X||^2 - 2<W, V'X> + <V'V, W W'>
 *       (synchronises when given; otherwise the call is stream-ordered)
 * NUMERIC when the objective is not finite. */
cox_status nmf_run(nmf_ctx *ctx, int32_t algo, int32_t iters, double eps, double *Vt, double *W, double *obj);

/* Measurement: HIP events around each launch of the two passes over X (phase 0:
 * W X', phase 1: V' X) while enabled; read returns the summed milliseconds and
 * the launch count.  Both synchronise. */
cox_status nmf_timing_enable(nmf_ctx *ctx, int32_t enable);
cox_status nmf_timing_read(nmf_ctx *ctx, int32_t phase, double *total_ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* NMF_H */
