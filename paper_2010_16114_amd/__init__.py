"""MI355X-native l1-regularised Cox regression by proximal gradient (ISTA).

A thin ctypes binding of libcoxhip (include/cox.h).  Every step of the method
runs in the library's HIP kernels; this module only marshals arguments.
PyTorch provides device memory and the stream.  There is no CPU fallback: if
the library is not built, importing the binding's entry points raises.

Matrices are column-major n x p: a torch tensor of shape (p, ldx) whose row j
is SNP column j (first n entries used).  Coefficients are (B, ptot) float32 with
ptot = p + q when q covariates are attached (the covariates last), linear
predictors (B, n).
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcoxhip.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "cox.h")
NMF_HEADER = os.path.join(os.path.dirname(_HERE), "include", "nmf.h")

X_F32, X_FP8_E4M3, X_INT8 = 0, 1, 2
MFMA_VARIANTS = 16  # COX_MFMA_VARIANTS: pipeline shapes of the X~' R pass (and the tuning arrays' length)
ETA_VARIANTS = 13  # COX_MFMA_ETA_VARIANTS: pipeline shapes of the eta update
MAX_COVARIATES = 64  # COX_MAX_COVARIATES
MAX_REFIT = 1024  # COX_MAX_REFIT
NOALLOC_MAX_COLS = 2097152  # COX_NOALLOC_MAX_COLS
OK, ERR_INVALID_ARG, ERR_OUT_OF_MEMORY, ERR_DEVICE, ERR_NUMERIC, ERR_NOT_CONVERGED, ERR_UNSUPPORTED = range(7)


class CoxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class _Matrix(ctypes.Structure):
    _fields_ = [("X", ctypes.c_void_p), ("xtype", ctypes.c_int32), ("n", ctypes.c_int64), ("p", ctypes.c_int64),
                ("ldx", ctypes.c_int64), ("col_center", ctypes.c_void_p), ("col_scale", ctypes.c_void_p)]


class RefitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("gtol", ctypes.c_double)]


class FitOpts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("tol", ctypes.c_double), ("lag", ctypes.c_int32),
                ("step", ctypes.c_double), ("warm_start", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("deterministic", ctypes.c_int32), ("eta_mode", ctypes.c_int32), ("poll", ctypes.c_int32),
                ("residual_bits", ctypes.c_int32), ("trace", ctypes.c_void_p)]


_lib = None


def declared_symbols() -> list[str]:
    """Function names declared by include/cox.h and include/nmf.h."""
    src = open(HEADER).read() + open(NMF_HEADER).read()
    return re.findall(r"^(?:cox_status|const char \*)\s*((?:cox|nmf)_\w+)\s*\(", src, flags=re.M)


def lib():
    """The loaded libcoxhip (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2010_16114_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64
    sig = {
        "cox_setup": [ctypes.POINTER(vp), ctypes.POINTER(_Matrix), vp, vp, i32, vp],
        "cox_destroy": [vp],
        "cox_last_error": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "cox_loss_grad": [vp, vp, i32, vp, vp],
        "cox_prox_step": [vp, vp, i32, vp, dbl, vp],
        "cox_prox_apply": [vp, vp, vp, i32, vp, dbl],
        "cox_fit_path": [vp, vp, i32, ctypes.POINTER(FitOpts), vp, vp, vp],
        "cox_fit_sequence": [vp, vp, i32, ctypes.POINTER(FitOpts), vp, vp, vp],
        "cox_set_covariates": [vp, vp, i64, i64],
        "cox_set_penalty_factors": [vp, vp],
        "cox_rank_path": [vp, vp, i32, vp, vp, vp, ctypes.POINTER(i64)],
        "cox_rank_path_noalloc": [vp, vp, i32, vp, vp, vp, ctypes.POINTER(i64)],
        "cox_refit": [vp, vp, i32, ctypes.POINTER(RefitOpts), vp, vp, vp, ctypes.POINTER(dbl),
                      ctypes.POINTER(i32)],
        "cox_lambda_max": [vp, ctypes.POINTER(dbl)],
        "cox_opnorm2": [vp, dbl, i32, u64, ctypes.POINTER(dbl), ctypes.POINTER(i32)],
        "cox_nll_forward": [vp, vp, i32, i32, vp],
        "cox_nll_backward": [vp, vp, i32, vp],
        "cox_timing_enable": [vp, i32],
        "cox_mfma_tuning": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), vp, vp],
        "cox_timing_read": [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
        "cox_timing_columns": [vp, ctypes.POINTER(i64)],
        "cox_device_bytes": [ctypes.POINTER(i64)],
        "nmf_setup": [ctypes.POINTER(vp), vp, i64, i64, i64, i32, vp],
        "nmf_destroy": [vp],
        "nmf_last_error": [vp, ctypes.c_char_p, ctypes.c_size_t],
        "nmf_run": [vp, i32, i32, dbl, vp, vp, vp],
        "nmf_timing_enable": [vp, i32],
        "nmf_timing_read": [vp, i32, ctypes.POINTER(dbl), ctypes.POINTER(i64)],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.cox_status_string.argtypes = [ctypes.c_int]
    L.cox_status_string.restype = ctypes.c_char_p
    _lib = L
    return L


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)



def device_bytes() -> int:
    """Device memory the library holds now (every context and call), in bytes."""
    v = ctypes.c_int64()
    st = lib().cox_device_bytes(ctypes.byref(v))
    if st != OK:
        raise CoxError(st, "cox_device_bytes")
    return v.value


class Cox:
    """One data set on the GPU (cox_setup).  X, center and scale are borrowed:
    this object keeps references to them for its lifetime."""

    def __init__(self, X, time, event, xtype: int | None = None, n: int | None = None, center=None, scale=None,
                 max_batch: int = 1, stream=None):
        import torch
        self._torch = torch
        if not X.is_cuda:
            raise ValueError("X must be a device tensor")
        if xtype is None:
            xtype = {torch.float32: X_F32, torch.int8: X_INT8, torch.uint8: X_FP8_E4M3,
                     torch.float8_e4m3fn: X_FP8_E4M3}[X.dtype]
        assert X.dim() == 2 and X.stride(1) == 1
        p, ldx = X.shape[0], X.stride(0)
        n = X.shape[1] if n is None else int(n)
        self.X, self.center, self.scale = X, center, scale
        self.n, self.p, self.max_batch, self.xtype = n, p, max_batch, xtype
        self.device = X.device
        self.stream = torch.cuda.current_stream(X.device) if stream is None else stream
        t = np.ascontiguousarray(time, dtype=np.float64)
        e = np.ascontiguousarray(event, dtype=np.int32)
        if t.shape != (n,) or e.shape != (n,):
            raise ValueError("time and event must have length n")
        m = _Matrix(X.data_ptr(), xtype, n, p, ldx, center.data_ptr() if center is not None else None,
                    scale.data_ptr() if scale is not None else None)
        h = ctypes.c_void_p()
        with torch.cuda.device(X.device):
            st = lib().cox_setup(ctypes.byref(h), ctypes.byref(m), _np_ptr(t), _np_ptr(e), max_batch,
                                 self.stream.cuda_stream)
        if st != OK:
            raise CoxError(st, f"cox_setup: {lib().cox_status_string(st).decode()}")
        self._h = h
        self.last_forward_key = None
        self.Z, self.q = None, 0

    # -- helpers
    def _check(self, st, what, allow=(OK,)):
        if st in allow:
            return st
        buf = ctypes.create_string_buffer(512)
        lib().cox_last_error(self._h, buf, 512)
        raise CoxError(st, f"{what}: {lib().cox_status_string(st).decode()} ({buf.value.decode()})")

    def _beta(self, beta):
        torch = self._torch
        assert beta.dtype == torch.float32 and beta.is_cuda and beta.is_contiguous()
        beta2 = beta.view(-1, self.ptot)
        return beta2, beta2.shape[0]

    @property
    def ptot(self) -> int:
        """Coefficients per vector: p, plus the attached covariates."""
        return self.p + self.q

    def close(self):
        if getattr(self, "_h", None):
            lib().cox_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points
    def set_covariates(self, Z):
        """Attach unpenalised covariates: Z a float32 device tensor of shape (q, ldz)
        whose row k is covariate k over the n subjects (None or q = 0 removes
        them).  Z is borrowed: this object keeps a reference."""
        if Z is None or Z.shape[0] == 0:
            self._check(lib().cox_set_covariates(self._h, None, 0, 0), "cox_set_covariates")
            self.Z, self.q = None, 0
            return
        torch = self._torch
        assert Z.dtype == torch.float32 and Z.is_cuda and Z.dim() == 2 and Z.stride(1) == 1
        self._check(lib().cox_set_covariates(self._h, Z.data_ptr(), Z.shape[0], Z.stride(0)), "cox_set_covariates")
        self.Z, self.q = Z, Z.shape[0]

    def set_penalty_factors(self, pf=None):
        """Penalty factors of the ptot columns (None: 1 for X's columns, 0 for covariates)."""
        if pf is None:
            self._check(lib().cox_set_penalty_factors(self._h, None), "cox_set_penalty_factors")
            return
        w = np.ascontiguousarray(np.asarray(pf, np.float64).reshape(-1))
        if w.shape != (self.ptot,):
            raise ValueError(f"pf must have ptot = {self.ptot} entries")
        self._check(lib().cox_set_penalty_factors(self._h, _np_ptr(w)), "cox_set_penalty_factors")

    def loss_grad(self, beta, want_grad: bool = True):
        """(-L(beta_b) for each b as numpy, gradient of -L as a (B, ptot) tensor or None)."""
        beta2, B = self._beta(beta)
        loss = np.empty(B, np.float64)
        grad = self._torch.empty_like(beta2) if want_grad else None
        st = lib().cox_loss_grad(self._h, beta2.data_ptr(), B, _np_ptr(loss),
                                 grad.data_ptr() if want_grad else None)
        self._check(st, "cox_loss_grad")
        return loss, grad

    def prox_step(self, beta, lambdas, step: float, want_obj: bool = True):
        beta2, B = self._beta(beta)
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lambdas, np.float64), (B,)))
        obj = np.empty(B, np.float64)
        st = lib().cox_prox_step(self._h, beta2.data_ptr(), B, _np_ptr(lam), float(step),
                                 _np_ptr(obj) if want_obj else None)
        self._check(st, "cox_prox_step")
        return obj if want_obj else None

    def prox_apply(self, beta, grad, lambdas, step: float):
        beta2, B = self._beta(beta)
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lambdas, np.float64), (B,)))
        st = lib().cox_prox_apply(self._h, beta2.data_ptr(), grad.data_ptr(), B, _np_ptr(lam), float(step))
        self._check(st, "cox_prox_apply")

    def fit_path(self, lambdas, max_iter: int = 1000, tol: float = 1e-5, lag: int = 10, step: float = 0.0,
                 beta=None, eta_mode: int = 0, poll: int = 16, residual_bits: int = 0, persistent: bool = False,
                 trace: bool = False, resume: bool = False):
        """ISTA for each lambda.  Returns (beta (B, ptot) tensor, iters, obj, status), and with
        trace=True a fifth item: the objective of every step, a (B, max_iter + 1) array (NaN past
        each lambda's last step).  resume=True continues the context's last fit_path (same B,
        lambdas, step, options) to max_iter in total, bit for bit as one call would."""
        torch = self._torch
        lam = np.ascontiguousarray(np.asarray(lambdas, np.float64).reshape(-1))
        B = lam.shape[0]
        warm = 2 if resume else int(beta is not None)
        if beta is None:
            beta = torch.zeros((B, self.ptot), dtype=torch.float32, device=self.device)
        beta2, Bb = self._beta(beta)
        assert Bb == B
        iters = np.zeros(B, np.int32)
        obj = np.zeros(B, np.float64)
        tr = np.full((B, int(max_iter) + 1), np.nan) if trace else None
        o = FitOpts(int(max_iter), float(tol), int(lag), float(step), int(warm), int(persistent), 1,
                    int(eta_mode), int(poll), int(residual_bits), tr.ctypes.data if trace else None)
        st = lib().cox_fit_path(self._h, _np_ptr(lam), B, ctypes.byref(o), beta2.data_ptr(), _np_ptr(iters),
                                _np_ptr(obj))
        self._check(st, "cox_fit_path", allow=(OK, ERR_NOT_CONVERGED))
        if trace:
            return beta2, iters, obj, st, tr
        return beta2, iters, obj, st

    def fit_sequence(self, lambdas, max_iter: int = 1000, tol: float = 1e-5, lag: int = 10, step: float = 0.0,
                     beta0=None, eta_mode: int = 0, poll: int = 16):
        """The sequential protocol: each lambda in turn, warm-started from the
        previous solution.  Returns (path (L, ptot) tensor, iters, obj, status)."""
        torch = self._torch
        lam = np.ascontiguousarray(np.asarray(lambdas, np.float64).reshape(-1))
        L = lam.shape[0]
        path = torch.zeros((L, self.ptot), dtype=torch.float32, device=self.device)
        if beta0 is not None:
            path[0] = beta0.reshape(-1)
        iters = np.zeros(L, np.int32)
        obj = np.zeros(L, np.float64)
        o = FitOpts(int(max_iter), float(tol), int(lag), float(step), int(beta0 is not None), 0, 1, int(eta_mode),
                    int(poll), 0, None)
        st = lib().cox_fit_sequence(self._h, _np_ptr(lam), L, ctypes.byref(o), path.data_ptr(), _np_ptr(iters),
                                    _np_ptr(obj))
        self._check(st, "cox_fit_sequence", allow=(OK, ERR_NOT_CONVERGED))
        return path, iters, obj, st

    def rank_path(self, path):
        """Section 6's ranking of a decreasing-lambda path (L, ptot): (entry row
        per column of X or -1, |coef| at entry, the entered columns in rank order)."""
        path2 = path.contiguous().view(-1, self.ptot)
        entry = np.zeros(self.p, np.int32)
        coef = np.zeros(self.p, np.float32)
        order = np.zeros(self.p, np.int64)
        ne = ctypes.c_int64()
        self._check(lib().cox_rank_path(self._h, path2.data_ptr(), path2.shape[0], _np_ptr(entry), _np_ptr(coef),
                                        _np_ptr(order), ctypes.byref(ne)), "cox_rank_path")
        return entry, coef, order[: ne.value]

    def rank_path_noalloc(self, path):
        """rank_path through cox_rank_path_noalloc: the same outputs, with the
        library's static device scratch instead of any allocation (at most
        NOALLOC_MAX_COLS columns)."""
        path2 = path.contiguous().view(-1, self.ptot)
        entry = np.zeros(self.p, np.int32)
        coef = np.zeros(self.p, np.float32)
        order = np.zeros(self.p, np.int64)
        ne = ctypes.c_int64()
        self._check(lib().cox_rank_path_noalloc(self._h, path2.data_ptr(), path2.shape[0], _np_ptr(entry),
                                                _np_ptr(coef), _np_ptr(order), ctypes.byref(ne)),
                    "cox_rank_path_noalloc")
        return entry, coef, order[: ne.value]

    def refit(self, cols, coef0=None, max_iter: int = 50, gtol: float = 1e-8):
        """Unpenalised Newton refit on columns `cols` of X plus the covariates.
        Returns (coef, se, pval, loglik, iters, status) over cols then covariates."""
        c = np.ascontiguousarray(np.asarray(cols, np.int64).reshape(-1))
        M = c.shape[0] + self.q
        coef = np.zeros(M, np.float64) if coef0 is None else np.ascontiguousarray(coef0, np.float64).copy()
        se = np.zeros(M, np.float64)
        pv = np.zeros(M, np.float64)
        L = ctypes.c_double()
        it = ctypes.c_int32()
        o = RefitOpts(int(max_iter), float(gtol))
        st = lib().cox_refit(self._h, _np_ptr(c) if c.size else None, c.shape[0], ctypes.byref(o), _np_ptr(coef),
                             _np_ptr(se), _np_ptr(pv), ctypes.byref(L), ctypes.byref(it))
        self._check(st, "cox_refit", allow=(OK, ERR_NOT_CONVERGED))
        return coef, se, pv, L.value, it.value, st

    def lambda_max(self) -> float:
        out = ctypes.c_double()
        self._check(lib().cox_lambda_max(self._h, ctypes.byref(out)), "cox_lambda_max")
        return out.value

    def opnorm2(self, tol: float = 1e-6, maxiter: int = 1000, seed: int = 95376):
        s2 = ctypes.c_double()
        it = ctypes.c_int32()
        st = lib().cox_opnorm2(self._h, float(tol), int(maxiter), int(seed) & (2**64 - 1), ctypes.byref(s2),
                               ctypes.byref(it))
        self._check(st, "cox_opnorm2")
        return s2.value, it.value

    def nll_forward(self, eta):
        """-L(eta_b) for eta of shape (B, n) (float32 or float64): a (B,) float64 tensor."""
        torch = self._torch
        assert eta.is_cuda and eta.is_contiguous() and eta.dtype in (torch.float32, torch.float64)
        eta2 = eta.view(-1, self.n)
        B = eta2.shape[0]
        loss = torch.empty(B, dtype=torch.float64, device=self.device)
        st = lib().cox_nll_forward(self._h, eta2.data_ptr(), int(eta.dtype == torch.float64), B, loss.data_ptr())
        self._check(st, "cox_nll_forward")
        self.last_forward_key = self.forward_key(eta)
        return loss

    PHASES = {"xtr": 0, "risk": 1, "eta": 2, "xtr_kernel": 3, "eta_kernel": 4, "cov": 5, "refit_hessian": 6,
              "refit_solve": 7, "persistent": 8}

    def mfma_tuning(self):
        """Pipeline shapes chosen by the autotuner and their tuning times (ms)."""
        xv, ev = ctypes.c_int32(), ctypes.c_int32()
        xm = np.zeros(MFMA_VARIANTS, np.float32)
        em = np.zeros(MFMA_VARIANTS, np.float32)
        self._check(lib().cox_mfma_tuning(self._h, ctypes.byref(xv), ctypes.byref(ev), _np_ptr(xm), _np_ptr(em)),
                    "cox_mfma_tuning")
        return {"xtr_variant": xv.value, "eta_variant": ev.value, "xtr_ms": xm.tolist(), "eta_ms": em.tolist()}

    def timing(self, enable: bool):
        self._check(lib().cox_timing_enable(self._h, int(enable)), "cox_timing_enable")

    def timing_read(self, phase: str):
        """(total milliseconds, number of timed launches) of a phase since timing(True)."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self._check(lib().cox_timing_read(self._h, self.PHASES[phase], ctypes.byref(ms), ctypes.byref(cnt)),
                    "cox_timing_read")
        return ms.value, cnt.value

    def timing_columns(self) -> int:
        """Columns of X read by the active-set eta updates since timing(True)."""
        v = ctypes.c_int64()
        self._check(lib().cox_timing_columns(self._h, ctypes.byref(v)), "cox_timing_columns")
        return v.value

    @staticmethod
    def forward_key(eta):
        return (eta.data_ptr(), eta._version, tuple(eta.shape), eta.dtype)

    def nll_backward(self, grad_loss, like):
        """-grad_loss_b * r_b at the eta of the last forward, shaped and typed like `like`."""
        torch = self._torch
        gl = grad_loss.to(torch.float64).contiguous().view(-1)
        out = torch.empty_like(like)
        st = lib().cox_nll_backward(self._h, gl.data_ptr(), gl.shape[0], out.data_ptr())
        self._check(st, "cox_nll_backward")
        return out


NMF_MULTIPLICATIVE, NMF_APG = 0, 1
NMF_MAX_RANK = 64  # NMF_MAX_RANK


class NMF:
    """Nonnegative matrix factorisation of one X on the GPU (nmf_setup, Section
    5.1).  X: float32 device tensor (m, ldx), row i of X in its first n entries;
    borrowed.  Factors are float64 device tensors Vt (r, m) and W (r, n)."""

    def __init__(self, X, r: int, n: int | None = None, stream=None):
        import torch
        self._torch = torch
        assert X.is_cuda and X.dtype == torch.float32 and X.dim() == 2 and X.stride(1) == 1
        self.X, self.m, self.ldx = X, X.shape[0], X.stride(0)
        self.n = X.shape[1] if n is None else int(n)
        self.r = int(r)
        self.stream = torch.cuda.current_stream(X.device) if stream is None else stream
        h = ctypes.c_void_p()
        st = lib().nmf_setup(ctypes.byref(h), X.data_ptr(), self.m, self.n, self.ldx, self.r,
                             self.stream.cuda_stream)
        if st != OK:
            raise CoxError(st, f"nmf_setup: {lib().cox_status_string(st).decode()}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().nmf_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, Vt, W, algo: int, iters: int, eps: float = 1e-10, want_obj: bool = True):
        """iters iterations in place on Vt (r, m) and W (r, n); returns f at the end (or None)."""
        torch = self._torch
        for t, shape in ((Vt, (self.r, self.m)), (W, (self.r, self.n))):
            assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous() and tuple(t.shape) == shape
        obj = ctypes.c_double()
        st = lib().nmf_run(self._h, int(algo), int(iters), float(eps), Vt.data_ptr(), W.data_ptr(),
                           ctypes.byref(obj) if want_obj else None)
        if st != OK:
            buf = ctypes.create_string_buffer(512)
            lib().nmf_last_error(self._h, buf, 512)
            raise CoxError(st, f"nmf_run: {lib().cox_status_string(st).decode()} ({buf.value.decode()})")
        return obj.value if want_obj else None

    def timing(self, enable: bool):
        st = lib().nmf_timing_enable(self._h, int(enable))
        if st != OK:
            raise CoxError(st, "nmf_timing_enable")

    def timing_read(self, phase: int):
        """(total ms, launches) of the W X' pass (0) or the V' X pass (1) since timing(True)."""
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        st = lib().nmf_timing_read(self._h, int(phase), ctypes.byref(ms), ctypes.byref(cnt))
        if st != OK:
            raise CoxError(st, "nmf_timing_read")
        return ms.value, cnt.value


from .autograd import BreslowNLL, CoxLinearNLL  # noqa: E402
