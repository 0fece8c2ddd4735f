"""Seeded synthetic inputs for the l1-Cox path (genotype-shaped and Gaussian).

Input generation only: nothing in this package computes a step of the Cox
method.  Both the oracle tests and the GPU tests/benchmark draw their inputs
from here, so that the two sides see identical data.

Recipes (they stand in for the UK Biobank genotypes of Section 6, which are not
available):

* minor-allele frequencies maf_j ~ U(0.05, 0.5) from numpy's PCG64;
* genotypes G_ij ~ Binomial(2, maf_j) from a counter hash (see ``genhash.c``):
  the numpy, C and HIP versions agree bit for bit, so a 200 GB matrix can be
  generated directly in device memory and any column regenerated on the host;
* standardisation constants from exact per-column counts: mu_j = mean, s_j =
  1/(population SD), 0 for a monomorphic column; both rounded to FP32 and used
  as such by every consumer;
* Gaussian X ~ N(0, 1) i.i.d. FP32 from PCG64 (the plain FP32 workload);
* true effects: k columns chosen without replacement, values N(0, 0.5^2);
* event times T ~ Exponential(rate = exp(eta_true)), censoring C ~
  Exponential(c) with c bisected until the realised censored fraction is within
  0.005 of the target; y = min(T, C), delta = 1[T <= C];
* optional discretisation to integer days 1..1000 (ties):
  day = clamp(ceil(1000 y / q99(y)), 1, 1000).
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_C_SRC = os.path.join(_HERE, "genhash.c")
_C_LIB = os.path.join(_HERE, "libcoxsim.so")
_HIP_SRC = os.path.join(_HERE, "genhash.hip")
_HIP_LIB = os.path.join(_HERE, "libcoxsim_hip.so")

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
FP8_E4M3_CODE = np.array([0x00, 0x38, 0x40], dtype=np.uint8)  # OCP E4M3: 0.0, 1.0, 2.0

SEED_BASE = 16114


# ----------------------------------------------------------------- builds

def build_host() -> str:
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", _C_LIB, _C_SRC], check=True)
    return _C_LIB


def build_device() -> str:
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-O3", "-shared", "-fPIC",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-o", _HIP_LIB, _HIP_SRC], check=True, stderr=subprocess.DEVNULL)
    return _HIP_LIB


_clib = None
_hlib = None


def _host_lib():
    global _clib
    if _clib is None:
        if not os.path.exists(_C_LIB) or os.path.getmtime(_C_LIB) < os.path.getmtime(_C_SRC):
            build_host()
        lib = ctypes.CDLL(_C_LIB)
        vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
        lib.coxsim_genotype_host.argtypes = [vp, i64, i64, i64, vp, u64, vp, ctypes.c_int]
        lib.coxsim_genotype_counts_host.argtypes = [vp, i64, i64, i64, vp, vp]
        _clib = lib
    return _clib


def _device_lib():
    global _hlib
    if _hlib is None:
        if not os.path.exists(_HIP_LIB):
            raise RuntimeError(f"{_HIP_LIB} is not built; run coxsim.build_device()")
        lib = ctypes.CDLL(_HIP_LIB)
        vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
        lib.coxsim_genotype_device.argtypes = [vp, i64, i64, i64, u64, vp, ctypes.c_int, vp, vp, vp]
        lib.coxsim_genotype_device.restype = ctypes.c_int
        _hlib = lib
    return _hlib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------ counter hash

def _mix64(z: np.ndarray) -> np.ndarray:
    z = (z ^ (z >> np.uint64(30))) * M1
    z = (z ^ (z >> np.uint64(27))) * M2
    return z ^ (z >> np.uint64(31))


def splitmix(x) -> np.ndarray:
    with np.errstate(over="ignore"):
        return _mix64(np.asarray(x, dtype=np.uint64) + GAMMA)


def maf_and_thresholds(p: int, seed: int):
    """maf_j ~ U(0.05, 0.5) and t_j = floor(maf_j 2^32) (uint32)."""
    maf = np.random.Generator(np.random.PCG64(seed)).uniform(0.05, 0.5, size=p)
    thr = np.floor(maf * 2.0**32).astype(np.uint64).astype(np.uint32)
    return maf, thr


def genotype_columns_numpy(n: int, cols, seed: int, thresholds) -> np.ndarray:
    """Reference (numpy) form of the counter hash: int8 array (len(cols), n)."""
    cols = np.asarray(cols, dtype=np.uint64)
    thr = np.asarray(thresholds, dtype=np.uint32)
    sk = splitmix(np.uint64(seed))
    i = np.arange(n, dtype=np.uint64)
    out = np.empty((len(cols), n), dtype=np.int8)
    with np.errstate(over="ignore"):
        for c, j in enumerate(cols):
            h = splitmix(((j << np.uint64(32)) | i) ^ sk)
            lo = (h & np.uint64(0xFFFFFFFF)).astype(np.uint32)
            hi = (h >> np.uint64(32)).astype(np.uint32)
            out[c] = (lo < thr[c]).astype(np.int8) + (hi < thr[c]).astype(np.int8)
    return out


def genotype_columns(n: int, cols, seed: int, thresholds, ldx: int | None = None, fmt: int = 0) -> np.ndarray:
    """Host (C, OpenMP) form: array (len(cols), ldx) of int8 counts or FP8 codes."""
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    thr = np.ascontiguousarray(thresholds, dtype=np.uint32)
    assert thr.shape == cols.shape
    ldx = n if ldx is None else ldx
    out = np.zeros((len(cols), ldx), dtype=np.int8)
    _host_lib().coxsim_genotype_host(_ptr(out), n, len(cols), ldx, _ptr(cols), int(seed), _ptr(thr), fmt)
    return out


def genotype_counts(G: np.ndarray, n: int):
    G = np.ascontiguousarray(G, dtype=np.int8)
    p, ldx = G.shape
    c1 = np.empty(p, np.int64)
    c2 = np.empty(p, np.int64)
    _host_lib().coxsim_genotype_counts_host(_ptr(G), n, p, ldx, _ptr(c1), _ptr(c2))
    return c1, c2


def standardisation(c1, c2, n: int):
    """FP32 (mu_j, s_j) from exact counts: x~ = (g - mu_j) s_j has mean 0 and
    population variance 1; s_j = 0 for a monomorphic column."""
    c1 = np.asarray(c1, np.float64)
    c2 = np.asarray(c2, np.float64)
    mu = (c1 + 2.0 * c2) / n
    var = (c1 + 4.0 * c2) / n - mu * mu
    var = np.where(var > 0, var, 0.0)
    sd = np.sqrt(var)
    with np.errstate(divide="ignore"):
        s = np.where(sd > 0, 1.0 / np.where(sd > 0, sd, 1.0), 0.0)
    return mu.astype(np.float32), s.astype(np.float32)


def genotype_device(n: int, p: int, seed: int, thresholds, fmt: int = 0, ldx: int | None = None, device="cuda"):
    """Generate G on the GPU (torch uint8 tensor of shape (p, ldx)) and return it
    with exact counts (c1, c2) as numpy arrays."""
    import torch
    ldx = n if ldx is None else ldx
    out = torch.zeros((p, ldx), dtype=torch.uint8, device=device)
    thr = torch.from_numpy(np.ascontiguousarray(thresholds, dtype=np.uint32).view(np.int32)).to(device)
    c1 = torch.empty(p, dtype=torch.int64, device=device)
    c2 = torch.empty(p, dtype=torch.int64, device=device)
    stream = torch.cuda.current_stream(out.device).cuda_stream
    rc = _device_lib().coxsim_genotype_device(out.data_ptr(), n, p, ldx, int(seed), thr.data_ptr(), fmt,
                                              c1.data_ptr(), c2.data_ptr(), stream)
    if rc:
        raise RuntimeError(f"coxsim_genotype_device failed ({rc})")
    return out, c1.cpu().numpy(), c2.cpu().numpy()


# ---------------------------------------------------------------- survival

def survival_times(eta_true: np.ndarray, censor_frac: float, rng: np.random.Generator, days: bool = False):
    """(y, delta) with T ~ Exp(rate exp(eta_true)) and independent Exp(c)
    censoring whose rate is bisected to the target censored fraction."""
    n = eta_true.shape[0]
    T = rng.standard_exponential(n) / np.exp(eta_true)
    V = rng.standard_exponential(n)
    lo, hi = -60.0, 60.0  # log c; censored iff V / c < T  <=>  V < c T
    logc = 0.0
    for _ in range(200):
        logc = 0.5 * (lo + hi)
        frac = float(np.mean(V < np.exp(logc) * T))
        if abs(frac - censor_frac) <= 0.005:
            break
        if frac < censor_frac:
            lo = logc
        else:
            hi = logc
    C = V / np.exp(logc)
    y = np.minimum(T, C)
    delta = (T <= C).astype(np.int32)
    if days:
        q = np.quantile(y, 0.99)
        y = np.clip(np.ceil(1000.0 * y / q), 1, 1000).astype(np.float64)
    return y.astype(np.float64), delta


@dataclasses.dataclass
class CoxData:
    """One synthetic problem.  X is column-major: arrays have shape (p, n)."""
    name: str
    n: int
    p: int
    kind: str                     # "gaussian" (X32 set) or "genotype" (G, mu, s set)
    time: np.ndarray
    event: np.ndarray
    beta_true: np.ndarray
    causal: np.ndarray
    seed: int
    X32: np.ndarray | None = None
    G: np.ndarray | None = None   # int8 counts, or None when generated on the device
    mu: np.ndarray | None = None
    s: np.ndarray | None = None
    thresholds: np.ndarray | None = None

    def standardized32(self) -> np.ndarray:
        """FP32 standardised genotypes (x~ = (g - mu) s in FP64, rounded to FP32)."""
        assert self.kind == "genotype" and self.G is not None
        out = np.empty(self.G.shape, np.float32)
        step = max(1, (1 << 24) // max(1, self.G.shape[1]))
        for j0 in range(0, self.G.shape[0], step):
            j1 = min(self.G.shape[0], j0 + step)
            out[j0:j1] = ((self.G[j0:j1].astype(np.float64) - self.mu[j0:j1, None].astype(np.float64))
                          * self.s[j0:j1, None].astype(np.float64))
        return out


def _effects(p: int, k: int, rng):
    causal = np.sort(rng.choice(p, size=k, replace=False))
    beta = np.zeros(p, np.float64)
    beta[causal] = rng.normal(0.0, 0.5, size=k)
    return causal, beta


def genotype_problem(n: int, p: int, k: int, censor_frac: float, seed: int, days: bool = False,
                     materialize: bool = True, name: str = "genotype") -> CoxData:
    """Genotype-shaped problem.  With materialize=False only the k causal columns
    are generated on the host (to draw the survival times) and the counts are
    left to whoever generates G (e.g. on the device)."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    _, thr = maf_and_thresholds(p, seed)
    causal, beta = _effects(p, k, rng)
    if materialize:
        G = genotype_columns(n, np.arange(p), seed, thr)
        c1, c2 = genotype_counts(G, n)
        mu, s = standardisation(c1, c2, n)
        Gc = G[causal]
    else:
        G, mu, s = None, None, None
        Gc = genotype_columns(n, causal, seed, thr[causal])
    c1c = (Gc == 1).sum(axis=1)
    c2c = (Gc == 2).sum(axis=1)
    muc, sc = standardisation(c1c, c2c, n)
    Xc = (Gc.astype(np.float64) - muc[:, None].astype(np.float64)) * sc[:, None].astype(np.float64)
    eta = Xc.T @ beta[causal]
    y, d = survival_times(eta, censor_frac, rng, days=days)
    return CoxData(name, n, p, "genotype", y, d, beta, causal, seed, G=G, mu=mu, s=s, thresholds=thr)


def covariate_block(n: int, q: int, seed: int) -> np.ndarray:
    """(q, n) FP32 covariates shaped like the application's unpenalised ones:
    row 0 a sex indicator (0/1, probability 1/2), rows 1.. standard normal
    stand-ins for principal components."""
    rng = np.random.Generator(np.random.PCG64(seed + 7))
    Z = np.empty((q, n), np.float32)
    if q > 0:
        Z[0] = (rng.random(n) < 0.5).astype(np.float32)
    if q > 1:
        Z[1:] = rng.standard_normal((q - 1, n), dtype=np.float32)
    return Z


def genotype_problem_with_covariates(n: int, p: int, k: int, q: int, censor_frac: float, seed: int,
                                     days: bool = False) -> tuple[CoxData, np.ndarray, np.ndarray]:
    """A genotype problem whose survival times also depend on q covariates
    (covariate_block) with effects gamma (sex 0.3, the others N(0, 0.2^2)).
    Returns (data, Z (q, n) FP32, gamma)."""
    d = genotype_problem(n, p, k, censor_frac, seed, days=days)
    Z = covariate_block(n, q, seed)
    rng = np.random.Generator(np.random.PCG64(seed + 11))
    gamma = np.concatenate([[0.3], rng.normal(0.0, 0.2, size=max(0, q - 1))])[:q]
    Gc = d.G[d.causal]
    Xc = (Gc.astype(np.float64) - d.mu[d.causal, None].astype(np.float64)) * d.s[d.causal, None].astype(np.float64)
    eta = Xc.T @ d.beta_true[d.causal] + Z.astype(np.float64).T @ gamma
    d.time, d.event = survival_times(eta, censor_frac, rng, days=days)
    return d, Z, gamma


def gaussian_problem(n: int, p: int, k: int, censor_frac: float, seed: int, name: str = "gaussian") -> CoxData:
    """X ~ N(0,1) i.i.d. FP32, not standardised."""
    rng = np.random.Generator(np.random.PCG64(seed + 1))
    X = np.random.Generator(np.random.PCG64(seed)).standard_normal(size=(p, n), dtype=np.float32)
    causal, beta = _effects(p, k, rng)
    eta = X[causal].astype(np.float64).T @ beta[causal]
    y, d = survival_times(eta, censor_frac, rng)
    return CoxData(name, n, p, "gaussian", y, d, beta, causal, seed, X32=X)


# ------------------------------------------------------------ the workloads

def config0(seed: int = SEED_BASE + 0) -> CoxData:
    """1,000 x 2,000 standardised genotypes, 10 effects, ~30% censored."""
    return genotype_problem(1000, 2000, 10, 0.30, seed, name="cox-geno-1000x2000")


def config1(n: int = 20000, p: int = 50000, seed: int = SEED_BASE + 1) -> CoxData:
    """20,000 x 50,000 Gaussian FP32, 50 effects, ~30% censored."""
    return gaussian_problem(n, p, 50, 0.30, seed, name=f"cox-gauss-{n}x{p}")


def config2(n: int = 100000, p: int = 10000, seed: int = SEED_BASE + 2) -> CoxData:
    """100,000 x 10,000 standardised genotypes, days 1..1000 (ties), ~30% censored."""
    return genotype_problem(n, p, 10, 0.30, seed, days=True, name=f"cox-geno-days-{n}x{p}")


def config3(n: int = 200000, p: int = 200000, seed: int = SEED_BASE + 3, materialize: bool = False) -> CoxData:
    """200,000 x 200,000 genotypes (stored FP8 E4M3), 200 effects, ~25% censored."""
    return genotype_problem(n, p, 200, 0.25, seed, materialize=materialize, name=f"cox-geno-fp8-{n}x{p}")


def config4(n: int = 400000, p: int = 500000, seed: int = SEED_BASE + 4, materialize: bool = False) -> CoxData:
    """400,000 x 500,000 genotypes (int8), 1,000 effects, 20% events."""
    return genotype_problem(n, p, 1000, 0.80, seed, materialize=materialize, name=f"cox-geno-int8-{n}x{p}")


def lambda_grid(lambda_max: float, B: int = 64, ratio: float = 0.01) -> np.ndarray:
    """B values log-spaced from lambda_max down to ratio * lambda_max."""
    if B == 1:
        return np.array([lambda_max], np.float64)
    return lambda_max * ratio ** (np.arange(B, dtype=np.float64) / (B - 1))
