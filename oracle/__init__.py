"""Plain FP64 CPU oracle for l1-regularised Cox regression (Section 5.3).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
GPU library is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product never does.  It
shares no code with the GPU path: the arithmetic lives in ``cox_oracle.c``
(plain double-precision loops, see its header for the passages it follows and
the readings it takes) and this module only marshals numpy arrays to it.

Matrices are column-major n x p, held as numpy arrays of shape (p, ldx) whose
row j is column j (the layout of Section 4.1's column-split MPIMatrix).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cox_oracle.c")
_SRC_NMF = os.path.join(_HERE, "nmf_oracle.c")
_LIB = os.path.join(_HERE, "libcoxoracle.so")

KIND_F64, KIND_F32, KIND_GENO = 0, 1, 2


def build() -> str:
    """Compile the oracle with gcc (IEEE semantics: no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-Wall", "-shared", "-fPIC", "-o", _LIB, _SRC, _SRC_NMF, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC), os.path.getmtime(_SRC_NMF)):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, dbl, u64, vp = ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p
    mat = [ctypes.c_int, vp, i64, i64, i64, vp, vp]
    lib.cox_oracle_order.argtypes = [i64, vp, vp, vp, vp]
    lib.cox_oracle_loglik.argtypes = [i64, vp, vp, vp, vp, vp]
    lib.cox_oracle_xbeta.argtypes = mat + [vp, vp]
    lib.cox_oracle_xtr.argtypes = mat + [vp, vp]
    lib.cox_oracle_soft_threshold.argtypes = [dbl, dbl]
    lib.cox_oracle_soft_threshold.restype = dbl
    lib.cox_oracle_loss_grad.argtypes = mat + [vp, vp, vp, vp, vp]
    lib.cox_oracle_lambda_max.argtypes = mat + [vp, vp, vp]
    lib.cox_oracle_opnorm2.argtypes = mat + [dbl, i32, u64, vp, vp]
    lib.cox_oracle_fit.argtypes = mat + [vp, vp, dbl, dbl, i32, dbl, i32, vp, vp, vp]
    lib.cox_oracle_fit_pf.argtypes = mat + [vp, vp, dbl, vp, dbl, i32, dbl, i32, vp, vp, vp]
    lib.cox_oracle_fit_hist.argtypes = mat + [vp, vp, dbl, dbl, i32, dbl, i32, vp, vp, vp, vp]
    lib.cox_oracle_newton.argtypes = mat + [vp, vp, vp, i64, vp, vp, i32, dbl, vp, vp]
    lib.cox_oracle_lambda_max_pf.argtypes = mat + [vp, vp, vp, dbl, vp, vp]
    lib.cox_oracle_rank_path.argtypes = [vp, i32, i64, i64, vp, vp, vp, vp]
    lib.nmf_oracle_objective.argtypes = [vp, i64, i64, i64, i32, vp, vp]
    lib.nmf_oracle_objective.restype = dbl
    lib.nmf_oracle_run.argtypes = [vp, i64, i64, i64, i32, i32, dbl, i32, vp, vp, vp]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


class Matrix:
    """A column-major n x p covariate matrix as the oracle reads it.

    kind KIND_F64 / KIND_F32: ``data`` holds the values.  KIND_GENO: ``data``
    holds int8 allele counts g and the value read is (g - mu_j) * s_j in FP64.
    """

    def __init__(self, kind: int, data: np.ndarray, n: int, mu=None, s=None):
        self.kind = kind
        self.data = np.ascontiguousarray(data)
        self.p, self.ldx = self.data.shape
        self.n = int(n)
        assert self.ldx >= self.n
        want = {KIND_F64: np.float64, KIND_F32: np.float32, KIND_GENO: np.int8}[kind]
        assert self.data.dtype == want, (self.data.dtype, want)
        self.mu = None if mu is None else np.ascontiguousarray(mu, dtype=np.float64)
        self.s = None if s is None else np.ascontiguousarray(s, dtype=np.float64)
        if kind == KIND_GENO:
            assert self.mu is not None and self.s is not None

    @classmethod
    def dense(cls, Xcm: np.ndarray, n: int | None = None):
        Xcm = np.asarray(Xcm)
        kind = KIND_F32 if Xcm.dtype == np.float32 else KIND_F64
        if kind == KIND_F64:
            Xcm = Xcm.astype(np.float64, copy=False)
        return cls(kind, Xcm, Xcm.shape[1] if n is None else n)

    @classmethod
    def genotype(cls, Gcm: np.ndarray, mu, s, n: int | None = None):
        Gcm = np.asarray(Gcm)
        return cls(KIND_GENO, Gcm.astype(np.int8, copy=False), Gcm.shape[1] if n is None else n, mu, s)

    def args(self):
        mu = None if self.mu is None else _ptr(self.mu)
        s = None if self.s is None else _ptr(self.s)
        return [self.kind, _ptr(self.data), self.n, self.p, self.ldx, mu, s]

    def to_dense64(self) -> np.ndarray:
        """The values the oracle reads, as an FP64 (p, n) array (small inputs)."""
        if self.kind == KIND_GENO:
            return (self.data[:, : self.n].astype(np.float64) - self.mu[:, None]) * self.s[:, None]
        return self.data[:, : self.n].astype(np.float64)


def _f64(a, n=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if n is not None:
        assert a.shape == (n,)
    return a


def _ev(event, n):
    e = np.ascontiguousarray(event, dtype=np.int32)
    assert e.shape == (n,)
    return e


def order(time):
    """Stable order by non-increasing time, and each position's tie group."""
    t = _f64(time)
    n = t.shape[0]
    o, gs, ge = (np.empty(n, np.int64) for _ in range(3))
    if _load().cox_oracle_order(n, _ptr(t), _ptr(o), _ptr(gs), _ptr(ge)):
        raise ValueError("non-finite time")
    return o, gs, ge


def loglik(eta, time, event):
    """Breslow log partial likelihood L(eta) and r = dL/deta (original order)."""
    e = _f64(eta)
    n = e.shape[0]
    t, ev = _f64(time, n), _ev(event, n)
    L = ctypes.c_double()
    r = np.empty(n, np.float64)
    if _load().cox_oracle_loglik(n, _ptr(e), _ptr(t), _ptr(ev), ctypes.byref(L), _ptr(r)):
        raise ValueError("bad input")
    return L.value, r


def xbeta(X: Matrix, beta):
    b = _f64(beta, X.p)
    out = np.empty(X.n, np.float64)
    if _load().cox_oracle_xbeta(*X.args(), _ptr(b), _ptr(out)):
        raise ValueError("bad matrix")
    return out


def xtr(X: Matrix, r):
    rr = _f64(r, X.n)
    out = np.empty(X.p, np.float64)
    if _load().cox_oracle_xtr(*X.args(), _ptr(rr), _ptr(out)):
        raise ValueError("bad matrix")
    return out


def soft_threshold(x: float, t: float) -> float:
    return _load().cox_oracle_soft_threshold(float(x), float(t))


def loss_grad(X: Matrix, time, event, beta):
    """(-L(beta), g = X'(I-P)delta), the gradient of L (not of -L)."""
    b = _f64(beta, X.p)
    t, ev = _f64(time, X.n), _ev(event, X.n)
    negL = ctypes.c_double()
    g = np.empty(X.p, np.float64)
    if _load().cox_oracle_loss_grad(*X.args(), _ptr(t), _ptr(ev), _ptr(b), ctypes.byref(negL), _ptr(g)):
        raise ValueError("bad input")
    return negL.value, g


def lambda_max(X: Matrix, time, event) -> float:
    t, ev = _f64(time, X.n), _ev(event, X.n)
    out = ctypes.c_double()
    if _load().cox_oracle_lambda_max(*X.args(), _ptr(t), _ptr(ev), ctypes.byref(out)):
        raise ValueError("bad input")
    return out.value


def opnorm2(X: Matrix, tol: float = 1e-6, maxiter: int = 1000, seed: int = 95376):
    """(||X||_2^2 by power iteration, steps taken); defaults of Section 4.3."""
    s2 = ctypes.c_double()
    it = ctypes.c_int32()
    if _load().cox_oracle_opnorm2(*X.args(), float(tol), int(maxiter), int(seed) & (2**64 - 1),
                                  ctypes.byref(s2), ctypes.byref(it)):
        raise ValueError("bad input")
    return s2.value, it.value


def fit(X: Matrix, time, event, lam: float, sigma: float, max_iter: int, tol: float = 0.0, lag: int = 10,
        beta0=None, pf=None):
    """ISTA for min -L + lam sum_j pf_j |beta_j| (pf None: every pf_j = 1).
    Returns (beta, objective trace f_0..f_K, K = steps taken, converged flag)."""
    t, ev = _f64(time, X.n), _ev(event, X.n)
    beta = np.zeros(X.p, np.float64) if beta0 is None else _f64(beta0, X.p).copy()
    trace = np.full(max_iter + 1, np.nan)
    it = ctypes.c_int32()
    lib = _load()
    if pf is None:
        rc = lib.cox_oracle_fit(*X.args(), _ptr(t), _ptr(ev), float(lam), float(sigma), int(max_iter),
                                float(tol), int(lag), _ptr(beta), _ptr(trace), ctypes.byref(it))
    else:
        w = _f64(pf, X.p)
        rc = lib.cox_oracle_fit_pf(*X.args(), _ptr(t), _ptr(ev), float(lam), _ptr(w), float(sigma),
                                   int(max_iter), float(tol), int(lag), _ptr(beta), _ptr(trace), ctypes.byref(it))
    if rc == -1:
        raise ValueError("bad input")
    if rc == -2:
        raise FloatingPointError("objective became non-finite")
    k = it.value
    return beta, trace[: k + 1], k, rc == 0


def fit_history(X: Matrix, time, event, lam: float, sigma: float, max_iter: int, tol: float = 0.0, lag: int = 10):
    """ISTA from beta = 0 as fit() (pf_j = 1), also returning every iterate.
    Returns (iterates (K + 1, p) with row k = beta_k, objective trace f_0..f_K, K)."""
    t, ev = _f64(time, X.n), _ev(event, X.n)
    beta = np.zeros(X.p, np.float64)
    trace = np.full(max_iter + 1, np.nan)
    hist = np.zeros((max_iter + 1, X.p), np.float64)
    it = ctypes.c_int32()
    rc = _load().cox_oracle_fit_hist(*X.args(), _ptr(t), _ptr(ev), float(lam), float(sigma), int(max_iter),
                                     float(tol), int(lag), _ptr(beta), _ptr(trace), _ptr(hist), ctypes.byref(it))
    if rc == -1:
        raise ValueError("bad input")
    if rc == -2:
        raise FloatingPointError("objective became non-finite")
    k = it.value
    return hist[: k + 1], trace[: k + 1], k


def newton(X: Matrix, time, event, cols, beta_fixed=None, beta_start=None, maxit: int = 100, gtol: float = 1e-10):
    """Unpenalised maximum partial likelihood over the columns ``cols`` (every
    other coefficient held at ``beta_fixed``, default 0) by Newton's method.
    Returns (beta over cols, inverse of -Hessian at it, Newton steps, converged)."""
    t, ev = _f64(time, X.n), _ev(event, X.n)
    c = np.ascontiguousarray(cols, dtype=np.int64)
    m = c.shape[0]
    bs = np.zeros(m, np.float64) if beta_start is None else _f64(beta_start, m).copy()
    bf = None if beta_fixed is None else _f64(beta_fixed, X.p)
    cov = np.empty((m, m), np.float64)
    it = ctypes.c_int32()
    rc = _load().cox_oracle_newton(*X.args(), _ptr(t), _ptr(ev), _ptr(c), m, None if bf is None else _ptr(bf),
                                   _ptr(bs), int(maxit), float(gtol), _ptr(cov), ctypes.byref(it))
    if rc == -1:
        raise ValueError("bad input")
    if rc == -2:
        raise np.linalg.LinAlgError("the negative Hessian is not positive definite")
    return bs, cov, it.value, rc == 0


def lambda_max_pf(X: Matrix, time, event, pf, gtol: float = 1e-10):
    """(lambda_max, beta over the unpenalised columns in increasing order) with
    penalty factors pf: the largest |g_j| / pf_j over penalised j at the
    unpenalised optimum over {j : pf_j = 0}."""
    t, ev = _f64(time, X.n), _ev(event, X.n)
    w = _f64(pf, X.p)
    out = ctypes.c_double()
    bu = np.zeros(max(1, int(np.count_nonzero(w == 0))), np.float64)
    rc = _load().cox_oracle_lambda_max_pf(*X.args(), _ptr(t), _ptr(ev), _ptr(w), float(gtol), ctypes.byref(out),
                                          _ptr(bu))
    if rc == -1:
        raise ValueError("bad input")
    if rc == -2:
        raise np.linalg.LinAlgError("the unpenalised fit failed")
    return out.value, bu[: int(np.count_nonzero(w == 0))]


# ---- nonnegative matrix factorisation (Section 5.1), nmf_oracle.c

NMF_MU, NMF_APG = 0, 1


def rank_path(path):
    """Section 6's ranking of a path of coefficient vectors (rows: the lambdas,
    decreasing; float32): (entry row per column, -1 if never nonzero;
    |coefficient| at entry; the entered columns in rank order)."""
    P = np.ascontiguousarray(path, dtype=np.float32)
    L, p = P.shape
    entry = np.empty(p, np.int32)
    coef = np.empty(p, np.float32)
    order = np.empty(p, np.int64)
    m = ctypes.c_int64()
    if _load().cox_oracle_rank_path(_ptr(P), L, p, p, _ptr(entry), _ptr(coef), _ptr(order), ctypes.byref(m)):
        raise ValueError("bad input")
    return entry, coef, order[: m.value]


def _nmf_args(X, Vt, W):
    X = np.ascontiguousarray(X, dtype=np.float32)
    m, n = X.shape
    Vt = np.ascontiguousarray(Vt, dtype=np.float64).copy()
    W = np.ascontiguousarray(W, dtype=np.float64).copy()
    r = Vt.shape[0]
    assert Vt.shape == (r, m) and W.shape == (r, n)
    return X, m, n, r, Vt, W


def nmf_objective(X, Vt, W) -> float:
    """||X - V W||_F^2 evaluated directly (X: (m, n) float32, Vt: (r, m), W: (r, n))."""
    X, m, n, r, Vt, W = _nmf_args(X, Vt, W)
    return _load().nmf_oracle_objective(_ptr(X), m, n, n, r, _ptr(Vt), _ptr(W))


def nmf_run(X, Vt0, W0, algo: int, iters: int, eps: float = 1e-10):
    """iters iterations of the multiplicative (algo 0) or APG (algo 1) update.
    Returns (Vt, W, objective before and after each iteration)."""
    X, m, n, r, Vt, W = _nmf_args(X, Vt0, W0)
    trace = np.empty(iters + 1, np.float64)
    if _load().nmf_oracle_run(_ptr(X), m, n, n, r, int(algo), float(eps), int(iters), _ptr(Vt), _ptr(W),
                              _ptr(trace)):
        raise ValueError("bad input")
    return Vt, W, trace
