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
