"""cox_fit_path with persistent = 1: every step of the lambda path in one
cooperative launch, phases separated by grid-wide barriers.

The persistent form runs the same per-workgroup code as the one-launch-per-
phase form, so the two must agree bit for bit: coefficients, steps taken,
final objectives and the objective trace.  Against the FP64 oracle the
iterates are held to the FP32 paths' bar (max|beta - beta_o| <= 1e-5
max|beta_o| and objective 1e-6 relative at the same step k from 0).  Cases:
the three storage types, B = 1..8 (every compiled batch width), lambdas that
stop early under the lag rule beside ones that run to max_iter, shapes with
ragged tails (n not a multiple of any tile, p not a multiple of a column
block), a problem large enough that every workgroup of the resident grid
handles several positions of each phase, and the requests the persistent form
does not serve (UNSUPPORTED before any device work).
"""
import numpy as np
import pytest

import coxsim
import oracle
from tests.gpu_helpers import device_problem, rel_beta_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402

BETA_TOL = 1e-5
OBJ_TOL = 1e-6


def _say(msg):
    print(f"[persistent] {msg}", flush=True)


@pytest.fixture(scope="module")
def c0():
    return coxsim.config0()


def _same(a, b):
    """Bit-identical results of two fit_path calls (beta, iters, obj, status, trace)."""
    ba, bb = a[0].cpu().numpy(), b[0].cpu().numpy()
    np.testing.assert_array_equal(ba.view(np.uint32), bb.view(np.uint32))
    np.testing.assert_array_equal(a[1], b[1])
    np.testing.assert_array_equal(a[2].view(np.uint64), b[2].view(np.uint64))
    assert a[3] == b[3]
    if len(a) > 4:
        np.testing.assert_array_equal(np.nan_to_num(a[4], nan=-1.0).view(np.uint64),
                                      np.nan_to_num(b[4], nan=-1.0).view(np.uint64))


@pytest.mark.parametrize("storage", ["f32", "int8", "fp8"])
def test_persistent_iterates_match_oracle(c0, storage):
    """1,000 x 2,000 at lambda = 0.5 lambda_max, compared with the oracle at
    k = 1, 10, 100, 200 and with the multi-launch form bit for bit."""
    _say(f"oracle problem, {storage}")
    cox, M = device_problem(c0, storage, ldx=(c0.n + 15) // 16 * 16, max_batch=8)
    lam = 0.5 * oracle.lambda_max(M, c0.time, c0.event)
    s2, _ = oracle.opnorm2(M)
    sigma = 1.0 / (2.0 * s2)
    for k in (1, 10, 100, 200):
        bo, tr, _, _ = oracle.fit(M, c0.time, c0.event, lam, sigma, max_iter=k)
        per = cox.fit_path([lam], max_iter=k, tol=0.0, step=sigma, persistent=True, trace=True)
        mul = cox.fit_path([lam], max_iter=k, tol=0.0, step=sigma, persistent=False, trace=True)
        _same(per, mul)
        beta, iters, obj, st, trace = per
        assert iters[0] == k and st == P.ERR_NOT_CONVERGED
        assert rel_beta_err(beta.cpu().numpy()[0], bo) <= BETA_TOL, k
        assert obj[0] == pytest.approx(tr[-1], rel=OBJ_TOL)
        np.testing.assert_allclose(trace[0], tr, rtol=OBJ_TOL)


@pytest.mark.parametrize("B", [1, 2, 3, 4, 5, 8])
def test_persistent_batches_and_early_stops(c0, B):
    """B lambdas from lambda_max down, lag-10 rule at 1e-7: the large lambdas
    stop early (some at once), the small ones later; every b against the
    multi-launch form bit for bit, and the stopping steps against the oracle's."""
    _say(f"B = {B}")
    cox, M = device_problem(c0, "fp8", ldx=(c0.n + 15) // 16 * 16, max_batch=8)
    lm = oracle.lambda_max(M, c0.time, c0.event)
    lams = lm * np.geomspace(1.01, 0.3, B) if B > 1 else np.array([0.6 * lm])
    s2, _ = oracle.opnorm2(M)
    sigma = 1.0 / (2.0 * s2)
    per = cox.fit_path(lams, max_iter=300, tol=1e-7, lag=10, step=sigma, persistent=True, trace=True)
    mul = cox.fit_path(lams, max_iter=300, tol=1e-7, lag=10, step=sigma, persistent=False, trace=True)
    _same(per, mul)
    beta, iters, obj, st, _ = per
    for b in range(B):
        bo, tr, ko, conv = oracle.fit(M, c0.time, c0.event, lams[b], sigma, max_iter=300, tol=1e-7, lag=10)
        assert iters[b] == ko, (b, iters[b], ko)
        assert rel_beta_err(beta.cpu().numpy()[b], bo) <= BETA_TOL, b
        assert obj[b] == pytest.approx(tr[-1], rel=OBJ_TOL)


@pytest.mark.parametrize("storage,n,p", [("f32", 1001, 37), ("int8", 3333, 1001), ("fp8", 9000, 70)])
def test_persistent_ragged_shapes(storage, n, p):
    d = coxsim.genotype_problem(n, p, 5, 0.3, 9100 + n, days=True)
    cox, M = device_problem(d, storage, ldx=(n + 15) // 16 * 16, max_batch=4)
    lm = oracle.lambda_max(M, d.time, d.event)
    lams = lm * np.array([0.9, 0.5, 0.2])
    s2, _ = oracle.opnorm2(M)
    sigma = 1.0 / (2.0 * s2)
    per = cox.fit_path(lams, max_iter=60, tol=0.0, step=sigma, persistent=True)
    mul = cox.fit_path(lams, max_iter=60, tol=0.0, step=sigma, persistent=False)
    _same(per, mul)
    for b in range(3):
        bo, tr, _, _ = oracle.fit(M, d.time, d.event, lams[b], sigma, max_iter=60)
        assert rel_beta_err(per[0].cpu().numpy()[b], bo) <= BETA_TOL
        assert per[2][b] == pytest.approx(tr[-1], rel=OBJ_TOL)


def test_persistent_zero_steps_and_no_events(c0):
    cox, M = device_problem(c0, "f32", max_batch=2)
    s2, _ = oracle.opnorm2(M)
    sigma = 1.0 / (2.0 * s2)
    lam = [0.5 * oracle.lambda_max(M, c0.time, c0.event)]
    per = cox.fit_path(lam, max_iter=0, tol=0.0, step=sigma, persistent=True, trace=True)
    mul = cox.fit_path(lam, max_iter=0, tol=0.0, step=sigma, persistent=False, trace=True)
    _same(per, mul)
    assert per[1][0] == 0 and not per[0].any()
    # no events: L = 0 and r = 0, so beta stays 0 and the objective is 0 at every step
    n, p = 500, 40
    X = torch.randn((p, n), device="cuda")
    cz = P.Cox(X, np.arange(n, dtype=float) + 1.0, np.zeros(n, np.int32), max_batch=2)
    per = cz.fit_path([1.0, 0.0], max_iter=15, tol=0.0, step=0.1, persistent=True)
    mul = cz.fit_path([1.0, 0.0], max_iter=15, tol=0.0, step=0.1, persistent=False)
    _same(per, mul)
    assert not per[0].any() and np.all(per[2] == 0.0)


def test_persistent_many_positions_per_workgroup():
    """20,000 x 50,000 Gaussian FP32 (4 GB): the column-sum phase alone has
    tens of thousands of workgroup positions, several per resident workgroup;
    30 steps from 0 at B = 2 against the multi-launch form bit for bit."""
    d = coxsim.config1()
    cox, M = device_problem(d, "f32", max_batch=2)
    lm = cox.lambda_max()
    s2, _ = cox.opnorm2(maxiter=30)
    sigma = 1.0 / (2.0 * s2)
    lams = [0.3 * lm, 0.1 * lm]
    per = cox.fit_path(lams, max_iter=30, tol=0.0, step=sigma, persistent=True, trace=True)
    mul = cox.fit_path(lams, max_iter=30, tol=0.0, step=sigma, persistent=False, trace=True)
    _same(per, mul)
    _say(f"20,000 x 50,000: nnz {np.count_nonzero(per[0].cpu().numpy(), axis=1)}, objective {per[2]}")


def test_persistent_unsupported_requests(c0):
    cox, M = device_problem(c0, "fp8", ldx=(c0.n + 15) // 16 * 16, max_batch=16)
    lam = np.full(16, 10.0)
    for kw, Bl in ((dict(), lam), (dict(eta_mode=1), lam[:2])):
        with pytest.raises(P.CoxError) as ei:
            cox.fit_path(Bl, max_iter=3, step=0.01, persistent=True, **kw)
        assert ei.value.status == P.ERR_UNSUPPORTED
    Z = torch.randn((2, c0.n), device="cuda")
    cox.set_covariates(Z)
    with pytest.raises(P.CoxError) as ei:
        cox.fit_path(lam[:2], max_iter=3, step=0.01, persistent=True)
    assert ei.value.status == P.ERR_UNSUPPORTED
    # X whose columns are not 16-byte aligned (ldx = n = 1000 is, n = 1001 is not)
    d = coxsim.genotype_problem(1001, 30, 3, 0.3, 77)
    cu, _ = device_problem(d, "int8", max_batch=2)
    with pytest.raises(P.CoxError) as ei:
        cu.fit_path([1.0], max_iter=3, step=0.01, persistent=True)
    assert ei.value.status == P.ERR_UNSUPPORTED
