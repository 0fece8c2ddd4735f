"""Shared set-up for the GPU tests: put one synthetic problem on the device in a
chosen storage format, and the matching oracle view of the same numbers."""
from __future__ import annotations

import numpy as np

import coxsim
import oracle


def device_problem(d: coxsim.CoxData, storage: str = "f32", ldx: int | None = None, max_batch: int = 1):
    """(Cox handle, oracle Matrix) for problem d.

    storage: "f32"  -- standardised FP32 X (genotypes) or the Gaussian X itself
             "int8" -- allele counts, standardised on the fly from mu, s
             "fp8"  -- the same counts as OCP FP8 E4M3 codes
    ldx: leading dimension (>= n); padding rows hold garbage-free zeros."""
    import torch
    import paper_2010_16114_amd as P
    n, p = d.n, d.p
    ldx = n if ldx is None else ldx
    if storage == "f32":
        Xh = d.X32 if d.kind == "gaussian" else d.standardized32()
        X = torch.zeros((p, ldx), dtype=torch.float32)
        X[:, :n] = torch.from_numpy(Xh)
        X = X.cuda()
        cox = P.Cox(X, d.time, d.event, n=n, max_batch=max_batch)
        M = oracle.Matrix.dense(Xh)
        return cox, M
    assert d.kind == "genotype"
    if storage == "int8":
        X = torch.zeros((p, ldx), dtype=torch.int8)
        X[:, :n] = torch.from_numpy(d.G)
        xtype = P.X_INT8
    else:
        X = torch.zeros((p, ldx), dtype=torch.uint8)
        X[:, :n] = torch.from_numpy(coxsim.FP8_E4M3_CODE[d.G])
        xtype = P.X_FP8_E4M3
    X = X.cuda()
    mu = torch.from_numpy(d.mu).cuda()
    s = torch.from_numpy(d.s).cuda()
    cox = P.Cox(X, d.time, d.event, xtype=xtype, n=n, center=mu, scale=s, max_batch=max_batch)
    M = oracle.Matrix.genotype(d.G, d.mu, d.s)
    return cox, M


def rel_beta_err(b, bo):
    b = np.asarray(b, np.float64)
    bo = np.asarray(bo, np.float64)
    scale = np.abs(bo).max()
    return np.abs(b - bo).max() / (scale if scale > 0 else 1.0)


def regenerate(d, mu, s, cols):
    """Oracle view of columns `cols` of a hash-generated genotype problem: the
    counts regenerated on the host with the problem's own standardisation."""
    cols = np.asarray(cols, np.int64)
    Gh = coxsim.genotype_columns(d.n, cols, d.seed, d.thresholds[cols])
    return oracle.Matrix.genotype(Gh, mu[cols], s[cols])


def restricted_iterates(cox, d, mu, s, lam, sigma, K, cand, say=print, rounds=4, margin=1e-4):
    """The FP64 oracle's ISTA iterates of the full problem, computed on a
    column subset.

    A column whose coefficient is 0 and whose gradient stays within
    [-lambda, lambda] is never moved by the proximal step, so ISTA on the
    columns `cand` reproduces the full problem's iterates exactly when every
    other column satisfies |g_j(beta_k)| <= lambda at each iterate k < K.  The
    oracle runs K steps from 0 on `cand` (regenerated from the counter hash)
    and the GPU evaluates the full gradient at each of its iterates (one
    batched cox_loss_grad); columns that come within `margin` of the threshold
    join `cand` and the run is repeated.  Returns (cols, iterates (K + 1,
    len(cols)), objective trace f_0..f_K)."""
    import torch
    cand = np.unique(np.asarray(cand, np.int64))
    for _ in range(rounds):
        M = regenerate(d, mu, s, cand)
        hist, trace, k = oracle.fit_history(M, d.time, d.event, lam, sigma, max_iter=K)
        assert k == K
        full = torch.zeros((K, d.p), dtype=torch.float32)
        full[:, torch.from_numpy(cand)] = torch.from_numpy(hist[:K].astype(np.float32))
        _, grad = cox.loss_grad(full.cuda())
        gmax = grad.abs().max(dim=0).values.cpu().numpy().astype(np.float64)  # max_k |g_j(beta_k)|
        gmax[cand] = 0.0
        extra = np.flatnonzero(gmax > lam * (1.0 - margin))
        say(f"restricted oracle on {cand.size} columns: {extra.size} more columns reach the threshold")
        if extra.size == 0:
            return cand, hist, trace
        cand = np.union1d(cand, extra)
    raise AssertionError("the candidate column set did not close")
