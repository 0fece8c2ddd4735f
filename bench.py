#!/usr/bin/env python3
"""Benchmark: l1-Cox proximal-gradient (ISTA) steps per second on one MI355X.

One "step" is one full iteration of the method for every coefficient vector of
the batch: eta update, risk-set sums and log likelihood, X~' r with the fused
soft-threshold, convergence check.  The timed region runs K steps from beta = 0
with every input already resident in HBM.  Prints one JSON line.

Workloads (synthetic, seeded; they stand in for the UK Biobank genotypes):
  geno-fp8-batched (default) : n = 400,000 subjects x p = 500,000 SNPs, allele
               counts stored as FP8 E4M3 codes (200 GB, generated in HBM),
               standardised on the fly; 1,000 true effects, 20% events; a path
               of B = 64 lambdas log-spaced from lambda_max to 0.01 lambda_max
               solved together; step 1/(2 ||X~||^2) with ||X~|| from 20 power
               steps; K steps from beta = 0.
  gauss-fp32 : n = 20,000 subjects x p = 50,000 covariates, X ~ N(0,1) FP32,
               50 true effects, ~30% censored, lambda = 0.3 lambda_max,
               step 1/(2 ||X||^2) by power iteration, 500 steps.
  refit      : Section 6's post-selection refit: n = 400,000 subjects, 333 SNP
               columns of an FP8 genotype matrix plus 11 unpenalised covariates,
               Newton's method with the exact Breslow Hessian to max |g| <= 1e-6
               (timed in Newton steps per second).
  nmf        : Section 5.1's NMF on its GPU shape, X 10,000 x 10,000 uniform
               FP32, rank 20 (--nmf-rank), multiplicative update (--nmf-algo 1:
               APG), 1000 iterations timed.
  geno-fp8-c3: n = 200,000 x p = 200,000 FP8 genotypes, one lambda =
               0.2 lambda_max, ISTA to a relative objective change below 1e-8
               over 10 steps; beside it the plain FP32 method on the same X
               standardised to FP32 (160 GB resident), unscaled, to the same
               tolerance, both checked against the FP64 oracle's objective.
  autograd-c2: n = 100,000 x p = 10,000 FP32 standardised genotypes with
               times in days (ties): milliseconds per forward + backward of
               the torch.autograd functions.
  dense-eta-c4: the dense X~ beta behind cox_loss_grad and warm starts, for
               B = 64 vectors over the default workload's 400,000 x 500,000 FP8
               genotypes: milliseconds per product on the matrix cores (three
               exact limb passes) and on the FP64 vector path.

The batched workload times K steps from beta = 0 `--repeats` times (default
3) and reports the median run; it also measures the HBM bandwidth the same
run sees (a torch copy and a torch reduction of a 4 GiB buffer), reads the
GPU clocks, and reports a per-step roofline: the algorithmic bytes of the
X~' R pass plus those of the eta update over the columns that changed
(counted on the device) over the median step time.

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
INT8_MFMA_PEAK_TOPS = 5000.0  # dense int8 matrix-core peak of the MI355X


def mfma_kernel_names(xtr_variant: int, eta_variant: int) -> tuple[str, str]:
    """Kernel names behind the matrix-core pipeline shapes the tuner kept:
    X~' R shapes 0-7 are `mfma_xtr_split_kernel`, 8-14 `mfma_xtr_lds_kernel`, 15
    that kernel with its last round split plus `xtr_tail_kernel`;
    eta shapes 0-1 are `mfma_eta_kernel`, 2-7 `mfma_eta_split_kernel`, and
    8-12 that kernel on one workgroup per compute unit plus `eta_fixup_kernel`."""
    xk = "mfma_xtr_split_kernel" if xtr_variant < 8 else "mfma_xtr_lds_kernel"
    if xtr_variant >= 15:
        xk += "+xtr_tail_kernel"
    if eta_variant < 2:
        ek = "mfma_eta_kernel"
    elif eta_variant < 8:
        ek = "mfma_eta_split_kernel"
    else:
        ek = "mfma_eta_split_kernel+eta_fixup_kernel"
    return xk, ek


def kernel_source_hash(files) -> str:
    """SHA-256 over the sources of a kernel, to tell whether a stored counter
    reading still describes the code that runs."""
    import hashlib

    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def stored_traffic(summary: str, sources, shape="all", per="launch") -> float | None:
    """HBM bytes per launch of a kernel, from a committed counter summary under
    profiles/ (FETCH_SIZE + WRITE_SIZE per dispatch, each scaled by what the
    same counter reads for a plain copy of known size), or None when there is
    none, the kernel's sources changed since it was taken, or it holds no
    figure for the pipeline shape that ran.  per = "column": bytes per changed
    column, for a kernel whose traffic grows with the columns it reads."""
    path = os.path.join(ROOT, "profiles", summary)
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        line = line.strip().lstrip("- ")
        if line.startswith(("traffic_bytes_per_", "source_sha256")) and ":" in line:
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != kernel_source_hash(sources):
        return None
    v = vals.get(f"traffic_bytes_per_{per}_{shape}")
    return float(v) if v is not None else None


MFMA_SOURCES = ("paper_2010_16114_amd/csrc/mfma.hip", "paper_2010_16114_amd/csrc/mfma.h")
GEMVT_SOURCES = ("paper_2010_16114_amd/csrc/gemvt.hip", "paper_2010_16114_amd/csrc/gemvt_dev.h",
                 "paper_2010_16114_amd/csrc/device_common.h",
                 "paper_2010_16114_amd/csrc/internal.h")


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


def hbm_probe(gib: float = 4.0, reps: int = 10) -> dict:
    """Measured HBM bandwidth of this GPU, taken in the same run as the
    workload: the median of `reps` device-to-device copies of a `gib` GiB
    buffer (bytes read + bytes written, per second) and of `reps` full
    reductions of it (bytes read per second), timed with events on torch's
    stream, on which both run."""
    import torch

    m = int(gib * (1 << 30)) // 4
    a = torch.ones(m, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    a.sum()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(2 * reps)]
    for k in range(reps):
        ev[k][0].record()
        b.copy_(a)
        ev[k][1].record()
    for k in range(reps, 2 * reps):
        ev[k][0].record()
        a.sum()
        ev[k][1].record()
    torch.cuda.synchronize()
    t_copy = float(np.median([s.elapsed_time(e) for s, e in ev[:reps]])) / 1e3
    t_read = float(np.median([s.elapsed_time(e) for s, e in ev[reps:]])) / 1e3
    del a, b
    torch.cuda.empty_cache()
    return {"copy_gbs": 2 * 4 * m / t_copy / 1e9, "read_gbs": 4 * m / t_read / 1e9, "buffer_bytes": 4 * m,
            "method": f"median of {reps} torch copies (read + write) and of {reps} torch sums (read) of a "
                      f"{gib:g} GiB buffer"}


def gpu_clocks() -> dict:
    """The GPU's clock levels as the kernel driver lists them before the
    workload (/sys/class/drm/card*/device/pp_dpm_sclk and pp_dpm_mclk, the
    active level marked '*'; an idle GPU sits at a low level), and the device's
    name; fields are left out when the files cannot be read."""
    import glob

    import torch

    prop = torch.cuda.get_device_properties(0)
    out = {"device": prop.name or getattr(prop, "gcnArchName", ""), "arch": getattr(prop, "gcnArchName", "")}
    for key in ("sclk", "mclk", "fclk"):
        for path in sorted(glob.glob(f"/sys/class/drm/card*/device/pp_dpm_{key}")):
            try:
                with open(path) as fh:
                    lines = fh.read().splitlines()
            except OSError:
                continue
            active = [l.strip() for l in lines if l.strip().endswith("*")]
            if active:
                out[key] = active[0]
                break
    return out


class ClockSampler:
    """Reads the GPU's active shader and memory clock levels (the '*' lines of
    /sys/class/drm/card*/device/pp_dpm_sclk and pp_dpm_mclk) every `period`
    seconds in a thread while the timed region runs, and reports the median,
    least and greatest MHz seen.  Reports nothing where the files cannot be
    read."""

    def __init__(self, period: float = 0.02):
        import glob

        self.period = period
        self.paths = {}
        for key in ("sclk", "mclk"):
            found = sorted(glob.glob(f"/sys/class/drm/card*/device/pp_dpm_{key}"))
            if found:
                self.paths[key] = found[0]
        self.counts = {key: {} for key in self.paths}
        self.samples = 0

    def _read(self):
        for key, path in self.paths.items():
            try:
                with open(path) as fh:
                    for line in fh:
                        line = line.strip()
                        if line.endswith("*"):
                            level = line.split(":", 1)[-1].strip(" *")
                            self.counts[key][level] = self.counts[key].get(level, 0) + 1
            except OSError:
                pass
        self.samples += 1

    def __enter__(self):
        import threading

        self._stop = threading.Event()

        def run():
            while not self._stop.is_set():
                self._read()
                self._stop.wait(self.period)

        self._thread = threading.Thread(target=run, daemon=True)
        if self.paths:
            self._thread.start()
        return self

    def __exit__(self, *exc):
        self._stop.set()
        if self.paths:
            self._thread.join()

    def summary(self) -> dict:
        out = {"samples": self.samples, "period_s": self.period}
        for key, c in self.counts.items():
            mhz = []
            for level, k in c.items():
                digits = level.lower().replace("mhz", "").strip()
                if digits.isdigit():
                    mhz += [int(digits)] * k
            if mhz:
                out[f"{key}_mhz"] = {"median": float(np.median(mhz)), "min": min(mhz), "max": max(mhz)}
        return out


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

    per = bool(args.persistent)
    log(f"warmup {args.warmup} steps ({'one persistent launch' if per else 'one launch per phase'})")
    cox.fit_path([lam], max_iter=args.warmup, tol=0.0, step=sigma, persistent=per)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    cox.timing(True)
    t0 = time.perf_counter()
    beta, iters, obj, _ = cox.fit_path([lam], max_iter=args.steps, tol=0.0, step=sigma, persistent=per)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    xtr_ms, xtr_n = cox.timing_read("xtr")
    risk_ms, risk_n = cox.timing_read("risk")
    eta_ms, eta_n = cox.timing_read("eta")
    xk_ms, xk_n = cox.timing_read("xtr_kernel")
    pk_ms, pk_n = cox.timing_read("persistent")
    cox.timing(False)
    elapsed = t1 - t0
    nnz = int((beta != 0).sum().item())
    log(f"{args.steps} steps in {elapsed:.3f} s; objective {obj[0]:.10g}; nnz {nnz}")

    # Algorithmic bytes of one launch of the column-sum kernel (B = 1): X once,
    # r once, one FP64 sum per column written.
    xtr_bytes = n * p * 4 + n * 4 + p * 8
    xtr_avg_s = xk_ms / max(xk_n, 1) / 1e3 if not per else pk_ms / 1e3 / args.steps
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
                               f"{args.steps} steps from beta=0" + (", one persistent launch" if per else ""),
                   "n": n, "p": p, "B": 1, "x_storage": "f32", "accumulate": "f64",
                   "eta": "active-set FP64 accumulator"},
        "phases_ms_per_step": {"xtr_prox": xtr_ms / max(xtr_n, 1), "risk": risk_ms / max(risk_n, 1),
                               "eta_update": eta_ms / max(eta_n, 1)},
        "persistent": per,
        "roofline": {"bound": "hbm", "kernel": "gemvt_sums_kernel (X~' r column sums)" if not per else
                     "fit_persistent_kernel (the whole step; X~' r bytes over the launch time per step)",
                     "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic(f"gemvt_sums_kernel_gauss_fp32_{n}x{p}_traffic.md", GEMVT_SOURCES),
                     "algorithmic_bytes_per_launch": xtr_bytes, "kernel_ms": 1e3 * xtr_avg_s,
                     "launches_timed": xk_n},
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
    k = int(max(2, min(600, budget_s / max(one / 2, 1e-6))))
    log(f"oracle: one step ~{one / 2:.2f} s; timing {k} steps")
    t0 = time.perf_counter()
    oracle.fit(M, d.time, d.event, lam, sigma, max_iter=k)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "lambda-iters/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first {k} ISTA steps from beta=0 on the full {d.n}x{d.p} FP32 X (FP64 arithmetic)"}


def bench_geno_batched(args):
    import torch

    import coxsim
    import paper_2010_16114_amd as P

    n, p, B = args.n or 400000, args.p or 500000, args.batch
    ldx = (n + 15) // 16 * 16
    probe = hbm_probe()
    clocks = gpu_clocks()
    log(f"HBM probe: copy {probe['copy_gbs']:.0f} GB/s, read {probe['read_gbs']:.0f} GB/s; clocks {clocks}")
    log(f"drawing survival times from the causal columns (n={n}, p={p})")
    d = coxsim.config4(n=n, p=p, materialize=False)
    log("generating FP8 genotype matrix in HBM")
    G, c1, c2 = coxsim.genotype_device(n, p, d.seed, d.thresholds, fmt=1, ldx=ldx)
    mu, sc = coxsim.standardisation(c1, c2, n)
    mu_d, sc_d = torch.from_numpy(mu).cuda(), torch.from_numpy(sc).cuda()
    torch.cuda.synchronize()
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=n, center=mu_d, scale=sc_d, max_batch=B)
    if args.covariates:
        # Section 6's unpenalised covariates (sex and principal components) beside the SNPs
        log(f"attaching {args.covariates} unpenalised covariates")
        Z = torch.from_numpy(coxsim.covariate_block(n, args.covariates, d.seed)).cuda()
        cox.set_covariates(Z)
    lmax = cox.lambda_max()
    s2, pit = cox.opnorm2(tol=1e-6, maxiter=args.power_steps)
    sigma = 1.0 / (2.0 * s2)
    lams = coxsim.lambda_grid(lmax, B, 0.01)
    log(f"lambda_max={lmax:.6g} ||X~||^2~{s2:.6g} ({pit} power steps) sigma={sigma:.4g}")
    log(f"warmup {args.warmup} steps (B={B}, residual in {args.residual_bits}-bit integers)")
    cox.fit_path(lams, max_iter=args.warmup, tol=0.0, step=sigma, residual_bits=args.residual_bits)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps from beta = 0, {args.repeats} times")
    cox.timing(True)
    runs = []
    with ClockSampler() as sampler:
        for rep in range(args.repeats):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            beta, iters, obj, _ = cox.fit_path(lams, max_iter=args.steps, tol=0.0, step=sigma,
                                               residual_bits=args.residual_bits)
            torch.cuda.synchronize()
            runs.append(time.perf_counter() - t0)
            log(f"repeat {rep}: {1e3 * runs[-1] / args.steps:.2f} ms per step")
    clocks["during_timed_region"] = sampler.summary()
    eta_cols = cox.timing_columns()
    xtr_ms, xtr_n = cox.timing_read("xtr")
    risk_ms, risk_n = cox.timing_read("risk")
    eta_ms, eta_n = cox.timing_read("eta")
    xk_ms, xk_n = cox.timing_read("xtr_kernel")
    ek_ms, ek_n = cox.timing_read("eta_kernel")
    cov_ms, cov_n = cox.timing_read("cov")
    cox.timing(False)
    elapsed = float(np.median(runs))
    nnz = (beta != 0).sum(dim=1).cpu().numpy()
    log(f"{args.steps} steps x {B} lambdas in {elapsed:.3f} s (median of {len(runs)}); "
        f"nnz per lambda {nnz.min()}..{nnz.max()}")
    bpad = (B + 15) // 16 * 16
    tuning = cox.mfma_tuning()
    xtr_kernel, eta_kernel = mfma_kernel_names(tuning["xtr_variant"], tuning["eta_variant"])
    # Algorithmic bytes of one launch of the matrix-core X~' R kernel: X once,
    # the residual limbs once, the raw column sums written once.
    limbs = 3 if args.residual_bits == 22 else 2
    xtr_bytes = n * p + limbs * bpad * n + B * p * 8
    xtr_avg = xk_ms / max(xk_n, 1) / 1e3
    achieved = xtr_bytes / xtr_avg / 1e9
    tops = 2.0 * n * p * limbs * bpad / xtr_avg / 1e12
    # A whole step's algorithmic bytes: the X~' R pass above, and the eta
    # update -- the changed columns of X (counted on the device), the update's
    # limbs, the FP64 eta read and written once.  The O((n + p) B) phases
    # (risk-set scans, quantisation, the proximal epilogue) move about 3 GB
    # more at 400,000 x 500,000 and are left out.
    cols_per_step = eta_cols / max(args.repeats * args.steps, 1)
    eta_bytes = n * cols_per_step + 3 * bpad * cols_per_step + 2 * 8 * B * n
    step_bytes = xtr_bytes + eta_bytes
    step_gbs = step_bytes / elapsed * args.steps / 1e9
    per_col = stored_traffic(f"mfma_xtr_kernel_geno_fp8_{n}x{p}_b{B}_traffic.md", MFMA_SOURCES,
                             f"eta_shape{tuning['eta_variant']}", per="column")
    eta_traffic = per_col * cols_per_step if per_col is not None and limbs == 3 else None
    res = {
        "metric": METRIC,
        "value": args.steps * B / elapsed,
        "unit": "lambda-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp8",
        "data": "synthetic",
        "config": {"workload": f"l1-Cox ISTA path, FP8 E4M3 genotype X n={n} p={p} (standardised on the fly), "
                               f"B={B} lambdas log-spaced lambda_max..0.01*lambda_max, {args.steps} steps from beta=0",
                   "n": n, "p": p, "B": B, "x_storage": "fp8_e4m3 allele counts", "x_bytes": n * p,
                   "gradient": f"int8 MFMA, residual rounded to {args.residual_bits}-bit integers in {limbs} "
                               f"int8 limbs, exact int32 accumulation",
                   "residual_bits": args.residual_bits,
                   "eta": "int8 MFMA over the changed columns, FP64 accumulator",
                   "covariates": args.covariates},
        "iters_per_s": args.steps / elapsed,
        "phases_ms_per_step": {"xtr_prox": xtr_ms / max(xtr_n, 1), "risk": risk_ms / max(risk_n, 1),
                               "eta_update": eta_ms / max(eta_n, 1),
                               "covariates": cov_ms / (args.steps * args.repeats) if args.covariates else 0.0},
        "kernels_ms_per_launch": {xtr_kernel: xk_ms / max(xk_n, 1), eta_kernel: ek_ms / max(ek_n, 1)},
        "repeats": args.repeats,
        "ms_per_step_runs": [1e3 * r / args.steps for r in runs],
        "hbm_probe": probe,
        "clocks": clocks,
        "roofline_step": {"bound": "hbm", "what": "one whole step: X~' R pass + eta update over the changed "
                                                  "columns, algorithmic bytes over the median step time",
                          "bytes_per_step": step_bytes, "xtr_bytes": xtr_bytes, "eta_bytes": eta_bytes,
                          "changed_columns_per_step": cols_per_step, "achieved": step_gbs, "peak": HBM_PEAK_GBS,
                          "unit": "GB/s", "frac": step_gbs / HBM_PEAK_GBS,
                          "frac_of_copy_probe": step_gbs / probe["copy_gbs"]},
        "roofline": {"bound": "hbm", "kernel": f"{xtr_kernel} (X~' R for B lambdas, shape {tuning['xtr_variant']})",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "frac_of_copy_probe": achieved / probe["copy_gbs"],
                     "frac_of_read_probe": achieved / probe["read_gbs"],
                     "traffic": stored_traffic(f"mfma_xtr_kernel_geno_fp8_{n}x{p}_b{B}_traffic.md", MFMA_SOURCES,
                                               f"shape{tuning['xtr_variant']}" + ("" if limbs == 3 else "_limbs2")),
                     "algorithmic_bytes_per_launch": xtr_bytes, "kernel_ms": 1e3 * xtr_avg, "launches_timed": xk_n,
                     "mfma_tops": tops, "mfma_frac_int8": tops / INT8_MFMA_PEAK_TOPS},
        "eta_kernel_roofline": {"bound": "hbm", "kernel": f"{eta_kernel} (eta += X[:, U] D for B lambdas, shape {tuning['eta_variant']})",
                                "achieved": eta_bytes / (ek_ms / max(ek_n, 1) / 1e3) / 1e9 if ek_n else None,
                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                "frac": eta_bytes / (ek_ms / max(ek_n, 1) / 1e3) / 1e9 / HBM_PEAK_GBS if ek_n else None,
                                "traffic": eta_traffic,
                                "algorithmic_bytes_per_launch": eta_bytes},
        "nnz_range": [int(nnz.min()), int(nnz.max())],
        "autotune": tuning,
    }
    if args.fp32_slice > 0:
        res["fp32_comparator"] = fp32_comparator(args, d, G, mu_d, sc_d, lams, sigma, n, p)
        res["speedup_vs_fp32"] = res["value"] / res["fp32_comparator"]["value_scaled"]
    del G
    torch.cuda.empty_cache()
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_geno(d, lams[-1], sigma, p)
    return res


def fp32_comparator(args, d, G, mu_d, sc_d, lams, sigma, n, p):
    """The plain FP32 method (one lambda per pass, FP32 standardised X) on the
    first p_s columns, K steps from beta = 0 at the largest and the smallest
    lambda of the path.  FP32 X of the full matrix (4 bytes per entry) does not
    fit in HBM; the step's passes over X grow linearly in p and its risk-set
    sums do not, so the measured time less the risk-set sums (timed with
    events) is scaled by p / p_s."""
    import torch

    import paper_2010_16114_amd as P

    ps = min(args.fp32_slice, p)
    log(f"FP32 comparator: standardising {ps} columns to FP32")
    X32 = standardise_fp8_to_fp32(G, mu_d, sc_d, ps, n)
    torch.cuda.synchronize()
    cox = P.Cox(X32, d.time, d.event, n=n, max_batch=1)
    rates, scaled = [], []
    for lam in (lams[0], lams[-1]):
        cox.fit_path([lam], max_iter=2, tol=0.0, step=sigma)
        torch.cuda.synchronize()
        cox.timing(True)
        t0 = time.perf_counter()
        cox.fit_path([lam], max_iter=args.steps, tol=0.0, step=sigma)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        risk_ms, _ = cox.timing_read("risk")
        cox.timing(False)
        rates.append(args.steps / dt)
        # the step's passes over X (X' r with its epilogue, the eta update) grow
        # with the columns; the risk-set sums do not
        risk_s = risk_ms / 1e3
        scaled.append(args.steps / ((dt - risk_s) * p / ps + risk_s))
    cox.close()
    del X32
    torch.cuda.empty_cache()
    r = float(np.mean(rates))
    rs = float(np.mean(scaled))
    log(f"FP32 comparator: {r:.1f} lambda-iters/s on {ps} columns -> {rs:.2f} scaled to {p}")
    return {"value_slice": r, "value_scaled": rs, "unit": "lambda-iters/s", "columns": ps,
            "method": "plain FP32 X (standardised), one lambda per pass, same step, "
                      f"{args.steps} steps from beta=0 at lambda_max and 0.01*lambda_max; the time of the step "
                      f"less its risk-set sums scaled by {p}/{ps} (the passes over X grow with the columns, the "
                      f"risk-set sums do not). The same-tolerance comparison without scaling is the geno-fp8-c3 "
                      f"workload"}


def cpu_baseline_geno(d, lam, sigma, p_full, p_sample: int = 8000, budget_s: float = 15.0):
    """The FP64 oracle on a column sample of the genotype workload: its steps
    from beta = 0 at the smallest lambda, timed on the host cores and scaled to
    the full column count (the oracle's step cost is linear in p)."""
    import coxsim
    import oracle

    cols = np.arange(p_sample)
    G = coxsim.genotype_columns(d.n, cols, d.seed, d.thresholds[cols])
    c1, c2 = coxsim.genotype_counts(G, d.n)
    mu, sc = coxsim.standardisation(c1, c2, d.n)
    M = oracle.Matrix.genotype(G, mu, sc)
    t0 = time.perf_counter()
    oracle.fit(M, d.time, d.event, lam, sigma, max_iter=1)
    one = time.perf_counter() - t0
    k = int(max(2, min(200, budget_s / max(one / 2, 1e-6))))
    log(f"oracle: one step on {p_sample} columns ~{one / 2:.2f} s; timing {k} steps")
    t0 = time.perf_counter()
    oracle.fit(M, d.time, d.event, lam, sigma, max_iter=k)
    dt = time.perf_counter() - t0
    return {"value": k / dt * p_sample / p_full, "unit": "lambda-iters/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"first {k} ISTA steps from beta=0 at lambda=0.01*lambda_max on the first {p_sample} of "
                      f"{p_full} columns (n={d.n}), scaled by {p_sample}/{p_full}"}


def standardise_fp8_to_fp32(G, mu_d, sc_d, ps, n, step=4096):
    """FP32 X~ = (g - mu) s of the first ps columns of FP8-coded counts G (on the device)."""
    import torch

    X32 = torch.empty((ps, G.shape[1]), dtype=torch.float32, device="cuda")
    for j0 in range(0, ps, step):
        j1 = min(ps, j0 + step)
        code = G[j0:j1].to(torch.int32)
        cnt = ((code >> 3) & 1) | ((code >> 5) & 2)  # FP8 E4M3 codes of 0, 1, 2 -> counts
        X32[j0:j1] = (cnt.to(torch.float32) - mu_d[j0:j1, None]) * sc_d[j0:j1, None]
        del code, cnt
    X32[:, n:] = 0.0
    return X32


def bench_geno_fp8_c3(args):
    """The precision workload: 200,000 x 200,000 genotypes stored as FP8 E4M3 codes
    (40 GB), one lambda = 0.2 lambda_max, ISTA from beta = 0 until the relative
    objective change over 10 steps is below 1e-8; beside it the plain FP32 method
    on the same X standardised to FP32 (160 GB, resident too), same step, same
    stopping rule.  Both results are checked against the FP64 oracle's objective
    at the returned beta (from the support columns regenerated on the host)."""
    import torch

    import coxsim
    import oracle
    import paper_2010_16114_amd as P

    n, p = args.n or 200000, args.p or 200000
    tol, lag = 1e-8, 10
    ldx = (n + 15) // 16 * 16
    probe = hbm_probe()
    d = coxsim.config3(n=n, p=p)
    log(f"generating FP8 genotype matrix {n}x{p} in HBM")
    G, c1, c2 = coxsim.genotype_device(n, p, d.seed, d.thresholds, fmt=1, ldx=ldx)
    mu, sc = coxsim.standardisation(c1, c2, n)
    mu_d, sc_d = torch.from_numpy(mu).cuda(), torch.from_numpy(sc).cuda()
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=n, center=mu_d, scale=sc_d)
    lam = 0.2 * cox.lambda_max()
    s2, pit = cox.opnorm2(maxiter=args.power_steps)
    sigma = 1.0 / (2.0 * s2)
    runs = {}
    for name, c in (("fp8", cox),):
        c.fit_path([lam], max_iter=3, tol=0.0, step=sigma)
        torch.cuda.synchronize()
        c.timing(True)
        t0 = time.perf_counter()
        beta, it, obj, st = c.fit_path([lam], max_iter=5000, tol=tol, lag=lag, step=sigma)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        xk_ms, xk_n = c.timing_read("xtr_kernel")
        c.timing(False)
        runs[name] = (beta.cpu().numpy()[0].astype(np.float64), int(it[0]), float(obj[0]), dt, xk_ms / max(xk_n, 1))
        log(f"{name}: {it[0]} steps to tolerance in {dt:.3f} s ({1e3 * dt / it[0]:.3f} ms per step), f = {obj[0]:.12g}")
    log("standardising to FP32 (160 GB)")
    X32 = standardise_fp8_to_fp32(G, mu_d, sc_d, p, n)
    torch.cuda.synchronize()
    c32 = P.Cox(X32, d.time, d.event, n=n)
    c32.fit_path([lam], max_iter=3, tol=0.0, step=sigma)
    torch.cuda.synchronize()
    c32.timing(True)
    t0 = time.perf_counter()
    beta, it, obj, st = c32.fit_path([lam], max_iter=5000, tol=tol, lag=lag, step=sigma)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    xk_ms, xk_n = c32.timing_read("xtr_kernel")
    c32.timing(False)
    runs["fp32"] = (beta.cpu().numpy()[0].astype(np.float64), int(it[0]), float(obj[0]), dt, xk_ms / max(xk_n, 1))
    log(f"fp32: {it[0]} steps to tolerance in {dt:.3f} s ({1e3 * dt / it[0]:.3f} ms per step), f = {obj[0]:.12g}")
    c32.close()
    del X32
    torch.cuda.empty_cache()
    # the oracle's FP64 objective at each returned beta, from its support columns
    b8, b32 = runs["fp8"][0], runs["fp32"][0]
    cols = np.union1d(np.flatnonzero(b8), np.flatnonzero(b32))
    Gh = coxsim.genotype_columns(n, cols, d.seed, d.thresholds[cols])
    M = oracle.Matrix.genotype(Gh, mu[cols], sc[cols])
    checks = {}
    for name in ("fp8", "fp32"):
        bv = runs[name][0]
        L, _ = oracle.loglik(oracle.xbeta(M, bv[cols]), d.time, d.event)
        f_or = -L + lam * np.abs(bv).sum()
        checks[name] = abs(runs[name][2] - f_or) / abs(f_or)
    k8, t8, ms8 = runs["fp8"][1], runs["fp8"][3], runs["fp8"][4]
    k32, t32, ms32 = runs["fp32"][1], runs["fp32"][3], runs["fp32"][4]
    x8 = n * p + 4 * n + 24 * p
    x32 = 4 * n * p + 4 * n + 24 * p
    res = {
        "metric": METRIC,
        "value": k8 / t8,
        "unit": "lambda-iters/s",
        "n_gpus": 1, "steps": k8, "warmup": 3, "ms_per_step": 1e3 * t8 / k8, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "fp8", "data": "synthetic",
        "config": {"workload": f"l1-Cox ISTA, FP8 E4M3 genotype X n={n} p={p}, lambda=0.2*lambda_max, B=1, "
                               f"from beta=0 to |f_k - f_k-{lag}|/(|f_k|+1) < {tol:g}", "n": n, "p": p, "B": 1},
        "time_to_tolerance_s": t8,
        "fp32_comparator": {"value": k32 / t32, "unit": "lambda-iters/s", "steps": k32, "time_to_tolerance_s": t32,
                            "ms_per_step": 1e3 * t32 / k32, "x_bytes": 4 * n * p,
                            "method": "plain FP32 X (the same counts standardised, 160 GB resident), same step and "
                                      "stopping rule, unscaled"},
        "speedup_at_equal_tolerance": t32 / t8,
        "precision": {"rel_objective_fp8_vs_fp32": abs(runs["fp8"][2] - runs["fp32"][2]) / abs(runs["fp32"][2]),
                      "rel_beta_fp8_vs_fp32": float(np.abs(b8 - b32).max() / max(np.abs(b32).max(), 1e-300)),
                      "nnz": [int(np.count_nonzero(b8)), int(np.count_nonzero(b32))],
                      "oracle_objective_at_returned_beta_rel_diff": checks},
        "roofline": {"bound": "hbm", "kernel": "gemvt_sums_kernel (X~' r column sums, FP8 X)",
                     "achieved": x8 / (ms8 / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": x8 / (ms8 / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": x8, "kernel_ms": ms8,
                     "fp32_kernel": {"achieved": x32 / (ms32 / 1e3) / 1e9, "kernel_ms": ms32,
                                     "algorithmic_bytes_per_launch": x32}},
        "hbm_probe": probe,
    }
    return res


def bench_autograd_c2(args):
    """The autograd workload: 100,000 x 10,000 standardised genotypes in FP32,
    survival times discretised to days (ties), time per forward + backward of
    CoxLinearNLL (beta -> -L(X~ beta), gradient -X~' r) and of BreslowNLL
    (eta -> -L(eta), gradient -r)."""
    import torch

    import coxsim
    import paper_2010_16114_amd as P

    d = coxsim.config2(n=args.n or 100000, p=args.p or 10000)
    X = torch.from_numpy(d.standardized32()).cuda()
    cox = P.Cox(X, d.time, d.event, max_batch=1)
    beta = torch.tensor(d.beta_true[None], dtype=torch.float32, device="cuda", requires_grad=True)
    K = args.steps

    def lin():
        loss = P.CoxLinearNLL.apply(beta, cox)
        loss.sum().backward()

    eta0 = (beta.detach() @ X).detach()
    eta = eta0.clone().requires_grad_(True)

    def bres():
        loss = P.BreslowNLL.apply(eta, cox)
        loss.sum().backward()

    out = {}
    for name, fn in (("linear", lin), ("breslow", bres)):
        for _ in range(max(args.warmup, 1)):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            fn()
        torch.cuda.synchronize()
        out[name] = 1e3 * (time.perf_counter() - t0) / K
        log(f"{name}: {out[name]:.4f} ms per forward + backward")
    xbytes = 4 * d.n * d.p
    return {
        "metric": "Cox negative log partial likelihood, forward + backward through torch.autograd",
        "value": out["linear"], "unit": "ms", "n_gpus": 1, "steps": K, "warmup": args.warmup,
        "ms_per_step": out["linear"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"autograd: CoxLinearNLL on standardised FP32 genotypes n={d.n} p={d.p}, "
                               f"times in days (ties), beta at the true effects", "n": d.n, "p": d.p},
        "breslow_on_eta_ms": out["breslow"],
        "roofline": {"bound": "hbm", "kernel": "forward + backward of CoxLinearNLL (two passes over X)",
                     "achieved": 2 * xbytes / (out["linear"] / 1e3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": 2 * xbytes / (out["linear"] / 1e3) / 1e9 / HBM_PEAK_GBS, "traffic": None},
    }


def bench_dense_eta_c4(args):
    """Dense X~ beta for B = 64 vectors over 400,000 x 500,000 FP8 genotypes, the
    pass behind cox_loss_grad, warm starts and the dense-eta ablation: three exact
    limb passes of the matrix-core eta update (one FP64-accurate product), against
    the FP64 vector passes of 8 vectors each (COXHIP_NO_MFMA=1).  Timed through
    cox_loss_grad without the gradient: the dense phase, its eta-update launches,
    and the losses of both forms."""
    import numpy as np
    import torch

    import coxsim
    import paper_2010_16114_amd as P

    n, p, B = args.n or 400000, args.p or 500000, args.batch
    ldx = (n + 15) // 16 * 16
    probe = hbm_probe()
    d = coxsim.config4(n=n, p=p, materialize=False)
    log("generating FP8 genotype matrix in HBM")
    G, c1, c2 = coxsim.genotype_device(n, p, d.seed, d.thresholds, fmt=1, ldx=ldx)
    mu, sc = coxsim.standardisation(c1, c2, n)
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=n, center=torch.from_numpy(mu).cuda(),
                scale=torch.from_numpy(sc).cuda(), max_batch=B)
    rng = np.random.default_rng(7)
    beta = np.zeros((B, p), np.float32)
    for b in range(B):  # 5% nonzero coefficients per vector (the cost does not depend on it)
        cols = rng.choice(p, p // 20, replace=False)
        beta[b, cols] = 0.01 * rng.standard_normal(cols.size)
    beta = torch.from_numpy(beta).cuda()
    out = {}
    for mode in ("mfma", "vector"):
        if mode == "vector":
            os.environ["COXHIP_NO_MFMA"] = "1"
        K = args.steps if mode == "mfma" else max(1, args.steps // 5)
        for _ in range(max(args.warmup, 1) if mode == "mfma" else 1):
            cox.loss_grad(beta, want_grad=False)
        cox.timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(K):
            loss, _ = cox.loss_grad(beta, want_grad=False)
        torch.cuda.synchronize()
        wall = 1e3 * (time.perf_counter() - t0) / K
        eta_ms, eta_n = cox.timing_read("eta")
        ek_ms, ek_n = cox.timing_read("eta_kernel")
        cox.timing(False)
        os.environ.pop("COXHIP_NO_MFMA", None)
        out[mode] = {"loss_grad_ms": wall, "dense_ms": eta_ms / max(eta_n, 1), "calls": K,
                     "eta_kernel_ms": ek_ms / ek_n if ek_n else None, "eta_kernel_launches": ek_n, "loss": loss}
        log(f"{mode}: {out[mode]['dense_ms']:.2f} ms per dense pass of {B} vectors ({wall:.2f} ms per call)")
    rel = float(np.max(np.abs(out["mfma"]["loss"] - out["vector"]["loss"]) / np.abs(out["vector"]["loss"])))
    tuning = cox.mfma_tuning()
    _, eta_kernel = mfma_kernel_names(0, tuning["eta_variant"])
    # algorithmic bytes of one dense product: X once, the FP64 coefficients read, eta written
    alg = n * p + 8 * B * p + 8 * B * n
    # one of its three eta-update launches: X once, the D limbs, eta read and written
    launch_bytes = n * p + 3 * ((B + 15) // 16 * 16) * ((p + 63) // 64 * 64) + 16 * B * n
    kms = out["mfma"]["eta_kernel_ms"]
    dense = out["mfma"]["dense_ms"]
    for m in out.values():
        m.pop("loss")
    return {
        "metric": "dense X~ beta for B vectors (cox_loss_grad, warm starts), ms per pass",
        "value": dense, "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": dense, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8", "data": "synthetic",
        "config": {"workload": f"dense X~ beta, FP8 E4M3 genotype X n={n} p={p}, B={B} vectors 5% nonzero, "
                               f"three exact 22-bit limb passes on the matrix cores", "n": n, "p": p, "B": B},
        "modes": out,
        "speedup_vs_vector": out["vector"]["dense_ms"] / dense,
        "loss_max_rel_diff_vs_vector": rel,
        "hbm_probe": probe,
        "roofline": {"bound": "hbm", "kernel": f"{eta_kernel} (one limb pass, every column selected)",
                     "achieved": launch_bytes / (kms / 1e3) / 1e9 if kms else None, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": launch_bytes / (kms / 1e3) / 1e9 / HBM_PEAK_GBS if kms else None,
                     "traffic": stored_traffic(f"mfma_eta_kernel_dense_geno_fp8_{n}x{p}_b{B}_traffic.md",
                                               MFMA_SOURCES, f"shape{tuning['eta_variant']}"),
                     "algorithmic_bytes_per_launch": launch_bytes, "kernel_ms": kms},
        "roofline_pass": {"what": "one dense product (three launches) against a single read of X",
                          "bytes": alg, "achieved": alg / (dense / 1e3) / 1e9,
                          "frac": alg / (dense / 1e3) / 1e9 / HBM_PEAK_GBS},
    }


FP64_VALU_PEAK_TFLOPS = 78.6


def bench_refit(args):
    """Section 6's post-selection refit at its size: n subjects, m SNPs of an FP8
    genotype matrix (standardised on the fly) plus q unpenalised covariates,
    Newton's method with the exact Breslow Hessian until max |g| <= gtol."""
    import torch

    import coxsim
    import paper_2010_16114_amd as P

    n, p, m, q = args.n or 400000, args.p or 4000, args.refit_cols, args.covariates or 11
    ldx = (n + 15) // 16 * 16
    log(f"drawing survival times (n={n}, p={p})")
    d = coxsim.genotype_problem(n, p, 40, 0.8, coxsim.SEED_BASE + 6, materialize=False)
    G, c1, c2 = coxsim.genotype_device(n, p, d.seed, d.thresholds, fmt=1, ldx=ldx)
    mu, sc = coxsim.standardisation(c1, c2, n)
    mu_d, sc_d = torch.from_numpy(mu).cuda(), torch.from_numpy(sc).cuda()
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=n, center=mu_d, scale=sc_d)
    Z = torch.from_numpy(coxsim.covariate_block(n, q, d.seed)).cuda()
    cox.set_covariates(Z)
    rng = np.random.default_rng(d.seed)
    extra = rng.choice(np.setdiff1d(np.arange(p), d.causal), m - d.causal.size, replace=False)
    cols = np.sort(np.concatenate([d.causal, extra]))
    log(f"refit on {m} SNPs + {q} covariates: warm-up")
    cox.refit(cols, max_iter=1)
    torch.cuda.synchronize()
    cox.timing(True)
    t0 = time.perf_counter()
    coef, se, pv, L, it, st = cox.refit(cols, gtol=args.refit_gtol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h_ms, h_n = cox.timing_read("refit_hessian")
    s_ms, s_n = cox.timing_read("refit_solve")
    cox.timing(False)
    elapsed = t1 - t0
    M = m + q
    log(f"{it} Newton steps in {elapsed:.3f} s (status {st}); {h_n} Hessians, {h_ms / max(h_n, 1):.2f} ms each")
    # the two Gram matrices of the information, M (M + 1) / 2 products per row at
    # 2 flops: over the n subjects, and over the G tie groups that hold events
    G = int(np.unique(d.time[d.event == 1]).size)
    flops = (n + G) * M * (M + 1)
    hess_s = h_ms / max(h_n, 1) / 1e3
    res = {
        "metric": "unpenalised Cox refit, Newton steps/s",
        "value": it / elapsed,
        "unit": "newton-steps/s",
        "n_gpus": 1,
        "steps": int(it),
        "warmup": 1,
        "ms_per_step": 1e3 * elapsed / max(it, 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"post-selection refit: n={n}, {m} SNPs (FP8 counts, standardised, gathered to "
                               f"FP32) + {q} covariates, Newton to max|g| <= {args.refit_gtol}",
                   "n": n, "columns": M, "event_groups": G, "status": int(st), "loglik": L},
        "phases_ms_per_step": {"hessian": h_ms / max(h_n, 1), "factor_solve": s_ms / max(it, 1)},
        "roofline": {"bound": "alu", "kernel": "the information matrix: its two Gram terms (gram_kernel) over the whole Hessian phase's time",
                     "achieved": flops / hess_s / 1e12, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": flops / hess_s / 1e12 / FP64_VALU_PEAK_TFLOPS, "traffic": None,
                     "flops_per_hessian": flops},
        "min_pval": float(pv.min()),
    }
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_refit(d, cols, mu, sc, Z.cpu().numpy(), n)
    return res


def cpu_baseline_refit(d, cols, mu, sc, Z, n, ns: int = 20000):
    """The FP64 oracle's Newton fit, as it stands, on the first ns subjects of the
    same columns: one Newton step timed on the host, scaled by ns / n."""
    import coxsim
    import oracle

    G = coxsim.genotype_columns(ns, cols, d.seed, d.thresholds[cols])
    X = np.vstack([(G.astype(np.float64) - mu[cols, None].astype(np.float64)) * sc[cols, None].astype(np.float64),
                   Z[:, :ns].astype(np.float64)])
    Mo = oracle.Matrix.dense(X)
    t0 = time.perf_counter()
    oracle.newton(Mo, d.time[:ns], d.event[:ns], np.arange(Mo.p), maxit=1, gtol=0.0)
    dt = time.perf_counter() - t0
    return {"value": ns / n / dt, "unit": "newton-steps/s", "cores": cpu_threads(), "kind": "oracle",
            "sample": f"one Newton step of the oracle on the first {ns} of {n} subjects, scaled by {ns}/{n}"}


# Section 5.1's single-GPU runtimes for 10,000 iterations at 10,000 x 10,000
# (the paper's own hardware; context only): seconds by (algorithm, r)
NMF_PAPER_1GPU_S = {(0, 20): 62, (0, 40): 72, (0, 60): 83, (1, 20): 61, (1, 40): 80, (1, 60): 85}


def bench_nmf(args):
    """Section 5.1's NMF on its GPU shape: X 10,000 x 10,000 uniform FP32, rank
    r, the multiplicative (0) or APG (1) update, K iterations timed."""
    import torch

    import paper_2010_16114_amd as P

    m = args.n or 10000
    n = args.p or 10000
    r, algo = args.nmf_rank, args.nmf_algo
    rng = np.random.default_rng(16114 + 7)
    Xh = rng.random((m, n), dtype=np.float32)
    X = torch.from_numpy(Xh).cuda()
    Vt0, W0 = rng.random((r, m)), rng.random((r, n))
    Vt, W = torch.from_numpy(Vt0).cuda(), torch.from_numpy(W0).cuda()
    nmf = P.NMF(X, r)
    log(f"NMF {m} x {n}, r = {r}, algorithm {algo}: {args.warmup} warm-up, {args.steps} timed iterations")
    nmf.run(Vt, W, algo, args.warmup, want_obj=False)
    torch.cuda.synchronize()
    nmf.timing(True)
    t0 = time.perf_counter()
    nmf.run(Vt, W, algo, args.steps, want_obj=False)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    w_ms, w_n = nmf.timing_read(0)
    v_ms, v_n = nmf.timing_read(1)
    nmf.timing(False)
    f = nmf.run(Vt, W, algo, 0)
    elapsed = t1 - t0
    # per pass over X: X once (4mn bytes), the factor tile reads and the split partials
    kms = max(w_ms / max(w_n, 1), v_ms / max(v_n, 1))
    wxt_name = ("the W X' pass (nmf_wxt_direct_kernel when the rows of X and W are 16-byte aligned, "
                "else nmf_wxt_kernel)")
    kname = wxt_name if w_ms / max(w_n, 1) >= v_ms / max(v_n, 1) else "nmf_vtx_kernel (V' X)"
    nbytes = 4.0 * m * n
    flops = 2.0 * m * n * r
    gbs = nbytes / (kms / 1e3) / 1e9
    tfs = flops / (kms / 1e3) / 1e12
    hbm = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
    alu = {"bound": "alu", "achieved": tfs, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
           "frac": tfs / FP64_VALU_PEAK_TFLOPS}
    roof = dict(hbm if hbm["frac"] >= alu["frac"] else alu)
    roof.update({"kernel": kname, "traffic": None, "kernel_ms": kms, "bytes_per_launch": nbytes,
                 "flops_per_launch": flops, "other_bound": alu if roof["bound"] == "hbm" else hbm})
    paper_s = NMF_PAPER_1GPU_S.get((algo, r))
    res = {
        "metric": "NMF iterations/s",
        "value": args.steps / elapsed,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"NMF {m} x {n} uniform FP32 X, r = {r}, "
                               f"{'multiplicative' if algo == 0 else 'APG'} update, factors FP64",
                   "m": m, "n": n, "r": r, "algorithm": algo},
        "phases_ms_per_step": {"wxt": w_ms / max(w_n, 1), "vtx": v_ms / max(v_n, 1)},
        "roofline": roof,
        "objective": f,
        "paper_context": None if paper_s is None else {"iters_per_s_on_the_papers_gpu": 10000 / paper_s},
    }
    if not args.no_cpu:
        import oracle
        t0 = time.perf_counter()
        oracle.nmf_run(Xh, Vt0, W0, algo, 1)
        dt = time.perf_counter() - t0
        k = max(1, min(10, int(15.0 / max(dt, 1e-3))))
        t0 = time.perf_counter()
        oracle.nmf_run(Xh, Vt0, W0, algo, k)
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": k / dt, "unit": "iters/s", "cores": cpu_threads(), "kind": "oracle",
                               "sample": f"{k} iterations of the oracle on the same X (the objective is evaluated "
                                         f"after each, as the oracle does)"}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=0, help="default: 50 (batched), 1000 (nmf) or 500")
    ap.add_argument("--warmup", type=int, default=-1, help="default: 3 (batched), 1 (dense-eta-c4) or 20")
    ap.add_argument("--workload", default="geno-fp8-batched",
                    choices=["geno-fp8-batched", "gauss-fp32", "refit", "nmf", "geno-fp8-c3", "autograd-c2",
                             "dense-eta-c4"])
    ap.add_argument("--nmf-rank", type=int, default=20, help="nmf workload: rank r")
    ap.add_argument("--nmf-algo", type=int, default=0, choices=[0, 1], help="nmf workload: 0 multiplicative, 1 APG")
    ap.add_argument("--refit-cols", type=int, default=333, help="refit workload: SNP columns refitted")
    ap.add_argument("--refit-gtol", type=float, default=1e-6, help="refit workload: Newton stop, max |gradient|")
    ap.add_argument("--batch", type=int, default=64)
    ap.add_argument("--repeats", type=int, default=3,
                    help="batched workload: timed runs of K steps from beta = 0; the median is reported")
    ap.add_argument("--power-steps", type=int, default=20)
    ap.add_argument("--residual-bits", type=int, default=22, choices=[22, 14],
                    help="batched workload: residual rounding of the matrix-core gradient pass "
                         "(22: three int8 limbs, the default; 14: two limbs)")
    ap.add_argument("--fp32-slice", type=int, default=31250,
                    help="columns of the FP32 comparator of the batched workload (0: skip)")
    ap.add_argument("--calibrate-copy-gb", type=float, default=0.0,
                    help="first copy a buffer of this many GB with torch (a plain copy kernel of known size, "
                         "for scaling the HBM counters)")
    ap.add_argument("--covariates", type=int, default=0,
                    help="batched workload: attach this many unpenalised covariates (sex + principal components)")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--p", type=int, default=0)
    ap.add_argument("--persistent", action="store_true",
                    help="gauss-fp32 workload: the whole fit in one persistent launch")
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
    if args.calibrate_copy_gb > 0:
        nbytes = int(args.calibrate_copy_gb * 1e9)
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = src.clone()
        torch.cuda.synchronize()
        log(f"copied {nbytes} bytes for counter calibration")
        del src, dst
        torch.cuda.empty_cache()
    batched = args.workload == "geno-fp8-batched"
    if args.steps <= 0:
        args.steps = {"geno-fp8-batched": 50, "nmf": 1000, "autograd-c2": 50, "dense-eta-c4": 10}.get(args.workload, 500)
    if args.warmup < 0:
        args.warmup = 3 if batched else (1 if args.workload == "dense-eta-c4" else 20)
    res = {"gauss-fp32": bench_gauss_fp32, "geno-fp8-batched": bench_geno_batched,
           "refit": bench_refit, "nmf": bench_nmf, "geno-fp8-c3": bench_geno_fp8_c3,
           "autograd-c2": bench_autograd_c2, "dense-eta-c4": bench_dense_eta_c4}[args.workload](args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
