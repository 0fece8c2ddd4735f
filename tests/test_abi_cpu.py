"""The C-ABI library loads, exports what include/cox.h declares, and rejects bad
arguments before any device work (no GPU needed: nothing here launches)."""
import ctypes

import numpy as np
import pytest

import paper_2010_16114_amd as P


def test_exports_every_declared_symbol():
    L = P.lib()
    syms = P.declared_symbols()
    assert len(syms) >= 12
    missing = [s for s in syms if not hasattr(L, s)]
    assert not missing


def test_status_strings():
    L = P.lib()
    assert L.cox_status_string(0) == b"ok"
    assert L.cox_status_string(1) == b"invalid argument"
    assert L.cox_status_string(5).startswith(b"maximum")
    assert L.cox_status_string(99) == b"unknown status"


def _setup(X=0x10000, xtype=0, n=10, p=3, ldx=10, center=None, scale=None, time=None, event=None, B=1,
           null_out=False):
    L = P.lib()
    t = np.arange(n, dtype=np.float64) + 1 if time is None else np.asarray(time, np.float64)
    e = np.ones(n, np.int32) if event is None else np.asarray(event, np.int32)
    m = P._Matrix(X, xtype, n, p, ldx, center, scale)
    h = ctypes.c_void_p()
    out = None if null_out else ctypes.byref(h)
    return L.cox_setup(out, ctypes.byref(m), P._np_ptr(t), P._np_ptr(e), B, None), h


@pytest.mark.parametrize("kw", [dict(null_out=True), dict(X=None), dict(xtype=3), dict(n=0, ldx=0),
                                dict(p=0), dict(ldx=9), dict(B=0), dict(B=65), dict(center=0x2000),
                                dict(time=[1, 2, np.nan] + [4] * 7), dict(event=[0, 1, 2] + [1] * 7),
                                dict(time=[1, np.inf] + [3] * 8)])
def test_setup_rejects_bad_arguments(kw):
    st, h = _setup(**kw)
    assert st == P.ERR_INVALID_ARG
    assert not h.value


def test_null_context_calls():
    L = P.lib()
    buf = ctypes.create_string_buffer(16)
    assert L.cox_last_error(None, buf, 16) == P.ERR_INVALID_ARG
    assert L.cox_destroy(None) == P.OK
    d = ctypes.c_double()
    assert L.cox_lambda_max(None, ctypes.byref(d)) == P.ERR_INVALID_ARG
    assert L.cox_loss_grad(None, None, 1, None, None) == P.ERR_INVALID_ARG
    assert L.cox_fit_path(None, None, 1, None, None, None, None) == P.ERR_INVALID_ARG
    assert L.cox_nll_forward(None, None, 0, 1, None) == P.ERR_INVALID_ARG
    assert L.cox_fit_sequence(None, None, 1, None, None, None, None) == P.ERR_INVALID_ARG
    assert L.cox_set_covariates(None, None, 0, 0) == P.ERR_INVALID_ARG
    assert L.cox_set_penalty_factors(None, None) == P.ERR_INVALID_ARG
    assert L.cox_rank_path(None, None, 1, None, None, None, None) == P.ERR_INVALID_ARG
    assert L.cox_rank_path_noalloc(None, None, 1, None, None, None, None) == P.ERR_INVALID_ARG
    assert L.cox_refit(None, None, 1, None, None, None, None, None, None) == P.ERR_INVALID_ARG
    assert L.nmf_run(None, 0, 1, 0.0, None, None, None) == P.ERR_INVALID_ARG
    assert L.nmf_destroy(None) == P.OK
    h = ctypes.c_void_p()
    assert L.nmf_setup(ctypes.byref(h), None, 10, 10, 10, 4, None) == P.ERR_INVALID_ARG and not h.value


def test_header_constants_match_binding():
    """The binding's enum values and array sizes are the ones include/cox.h declares."""
    import re
    text = open(P.HEADER).read()
    assert int(re.search(r"#define COX_MFMA_VARIANTS (\d+)", text).group(1)) == P.MFMA_VARIANTS
    assert int(re.search(r"#define COX_MFMA_ETA_VARIANTS (\d+)", text).group(1)) == P.ETA_VARIANTS
    assert int(re.search(r"#define COX_MAX_COVARIATES (\d+)", text).group(1)) == P.MAX_COVARIATES
    assert int(re.search(r"#define COX_MAX_REFIT (\d+)", text).group(1)) == P.MAX_REFIT
    assert int(re.search(r"#define COX_NOALLOC_MAX_COLS (\d+)", text).group(1)) == P.NOALLOC_MAX_COLS
    ntext = open(P.NMF_HEADER).read()
    assert int(re.search(r"#define NMF_MAX_RANK (\d+)", ntext).group(1)) == P.NMF_MAX_RANK
    assert re.search(r"NMF_APG\s*=\s*(\d+)", ntext).group(1) == str(P.NMF_APG)
    assert re.search(r"COX_X_FP8_E4M3\s*=\s*(\d+)", text).group(1) == str(P.X_FP8_E4M3)
    assert re.search(r"COX_X_INT8\s*=\s*(\d+)", text).group(1) == str(P.X_INT8)


def test_fit_opts_layout_matches_header():
    """The binding's cox_fit_opts has the header's fields, in order."""
    import re
    text = open(P.HEADER).read()
    body = text.split("} cox_fit_opts;")[0].rsplit("typedef struct {", 1)[1]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"\b(?:int32_t|double)\s*\*?\s*(\w+);", body)
    assert fields == [f[0] for f in P.FitOpts._fields_]
    # the fields the boundary's specification names come first, in its order
    assert fields[:7] == ["max_iter", "tol", "lag", "step", "warm_start", "persistent", "deterministic"]
    assert ctypes.sizeof(P.FitOpts) == 64
