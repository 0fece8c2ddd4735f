#!/usr/bin/env python3
"""Benchmark: l1-Cox proximal-gradient (ISTA) steps per second on one MI355X.

One "step" is one full iteration of the method for every coefficient vector of
the batch: eta update, risk-set sums and log likelihood, X~' r with the fused
soft-threshold, convergence check.  The timed region runs K steps from beta = 0
with every input already resident in HBM.  Prints one JSON line.

Workloads (synthetic, seeded; they stand in for the UK Biobank genotypes):
  gauss-fp32 : n = 20,000 subjects x p = 50,000 covariates, X ~ N(0,1) FP32,
               50 true effects, ~30% censored, lambda = 0.3 lambda_max,
               step 1/(2 ||X||^2) by power iteration, 500 steps.

The oracle (plain FP64 C) is timed on the host cores on a bounded sample of
the same workload as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Cox prox-grad iters/s + HBM GB/s, FP8-X batched vs plain FP32, equal tolerance"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def bench_gauss_fp32(args):
    import torch

    import coxsim
    import paper_2010_16114_amd as P

    n, p = args.n or 20000, args.p or 50000
    log(f"generating Gaussian FP32 problem n={n} p={p}")
    d = coxsim.config1(n=n, p=p)
    X = torch.from_numpy(d.X32).cuda()
    torch.cuda.synchronize()
    cox = P.Cox(X, d.time, d.event)
    lmax = cox.lambda_max()
    lam = 0.3 * lmax
    s2, pit = cox.opnorm2()
    sigma = 1.0 / (2.0 * s2)
    log(f"lambda_max={lmax:.6g} ||X||^2={s2:.6g} ({pit} power steps), sigma={sigma:.4g}")

    log(f"warmup {args.warmup} steps")
    cox.fit_path([lam], max_iter=args.warmup, tol=0.0, step=sigma)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    cox.timing(True)
    t0 = time.perf_counter()
    beta, iters, obj, _ = cox.fit_path([lam], max_iter=args.steps, tol=0.0, step=sigma)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xtr_ms, xtr_n = cox.timing_read("xtr")
    risk_ms, risk_n = cox.timing_read("risk")
    eta_ms, eta_n = cox.timing_read("eta")
    cox.timing(False)
    elapsed = t1 - t0
    nnz = int((beta != 0).sum().item())
    log(f"{args.steps} steps in {elapsed:.3f} s; objective {obj[0]:.10g}; nnz {nnz}")

    # Algorithmic bytes of one X~' r launch (B = 1): X once, r once, and the FP64
    # iterate read and written with its change coefficient written.
    xtr_bytes = n * p * 4 + n * 4 + p * 8 * 3
    xtr_avg_s = xtr_ms / max(xtr_n, 1) / 1e3
    achieved = xtr_bytes / xtr_avg_s / 1e9
    steps_per_s = args.steps / elapsed
    res = {
        "metric": METRIC,
        "value": steps_per_s,
        "unit": "lambda-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"l1-Cox ISTA, Gaussian FP32 X n={n} p={p}, lambda=0.3*lambda_max, B=1, "
                               f"{args.steps} steps from beta=0",
                   "n": n, "p": p, "B": 1, "x_storage": "f32", "accumulate": "f64",
                   "eta": "active-set FP64 accumulator"},
        "phases_ms_per_step": {"xtr_prox": xtr_ms / max(xtr_n, 1), "risk": risk_ms / max(risk_n, 1),
                               "eta_update": eta_ms / max(eta_n, 1)},
        "roofline": {"bound": "hbm", "kernel": "gemvt_kernel (X~' r + prox)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_launch": xtr_bytes},
        "objective": float(obj[0]),
        "nnz": nnz,
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_gauss(d, lam, sigma)
    return res


def cpu_baseline_gauss(d, lam, sigma, budget_s: float = 15.0):
    """The FP64 oracle, as it stands, on the same X: a few ISTA steps from
    beta = 0 timed on the host cores, in lambda-iterations per second."""
    import oracle

    M = oracle.Matrix.dense(d.X32)
    t0 = time.perf_counter()
    oracle.fit(M, d.time, d.event, lam, sigma, max_iter=1)
    one = time.perf_counter() - t0
    k = int(max(2, min(100, budget_s / max(one / 2, 1e-6))))
    log(f"oracle: one step ~{one / 2:.2f} s; timing {k} steps")
    t0 = time.perf_counter()
    oracle.fit(M, d.time, d.event, lam, sigma, max_iter=k)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "lambda-iters/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first {k} ISTA steps from beta=0 on the full {d.n}x{d.p} FP32 X (FP64 arithmetic)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="gauss-fp32", choices=["gauss-fp32"])
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--p", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (SNP-sharding is a design, "
              "not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    res = {"gauss-fp32": bench_gauss_fp32}[args.workload](args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
