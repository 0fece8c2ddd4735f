"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (stated by the method's acceptance bar for the FP32 paths):
relative objective <= 1e-6 and max|beta - beta_oracle| <= 1e-5 max|beta_oracle|
at the same step k from the same start.  Quantities that the GPU computes in
FP64 end to end (the log likelihood at a given FP32 beta) are held to 1e-12.
Gradients, which pass through the FP32 residual and an FP32 output, to
1e-6 of their largest entry.
"""
import ctypes

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


@pytest.fixture(scope="module")
def c0():
    return coxsim.config0()


def _step(M, d):
    s2, _ = oracle.opnorm2(M)
    return 1.0 / (2.0 * s2)


def test_fp8_codes_decode_exactly():
    # one FP8 code per column, placed in row 0; at beta = 0 the gradient of -L
    # is -x_0j r_0, so grad_j / (-r_0) must equal the code's value.
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], dtype=np.uint8)
    n, p = 64, len(codes)
    Xh = np.zeros((p, n), np.uint8)
    Xh[:, 0] = codes
    t = np.arange(n, 0, -1).astype(float)
    e = np.ones(n, np.int32)
    cox = P.Cox(torch.from_numpy(Xh).cuda(), t, e, xtype=P.X_FP8_E4M3)
    _, grad = cox.loss_grad(torch.zeros((1, p), device="cuda"))
    _, r = oracle.loglik(np.zeros(n), t, e)
    want = torch.from_numpy(codes).view(torch.float8_e4m3fn).float().numpy()
    got = grad.cpu().numpy()[0] / (-r[0])
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=0)


@pytest.mark.parametrize("storage", ["f32", "int8", "fp8"])
def test_loss_grad(c0, storage):
    rng = np.random.default_rng(0)
    beta = np.zeros((3, c0.p), np.float32)
    beta[1, c0.causal] = c0.beta_true[c0.causal]
    beta[2] = (0.05 * rng.standard_normal(c0.p)).astype(np.float32)
    cox, M = device_problem(c0, storage, max_batch=3)
    loss, grad = cox.loss_grad(torch.from_numpy(beta).cuda())
    grad = grad.cpu().numpy()
    for b in range(3):
        negL, g = oracle.loss_grad(M, c0.time, c0.event, beta[b].astype(np.float64))
        assert loss[b] == pytest.approx(negL, rel=1e-12)
        assert np.abs(grad[b] + g).max() <= 1e-6 * np.abs(g).max()


@pytest.mark.parametrize("n,p,ldx,ties", [(1001, 37, 1001, False), (1001, 37, 1024, True), (2500, 16, 2500, True),
                                          (4099, 53, 4112, False), (1, 3, 1, False), (9000, 5, 9008, True)])
def test_ragged_shapes_f32(n, p, ldx, ties):
    d = coxsim.genotype_problem(n, p, min(3, p), 0.3, 77 + n, days=ties)
    cox, M = device_problem(d, "f32", ldx=ldx)
    beta = (0.1 * np.random.default_rng(n).standard_normal(p)).astype(np.float32)
    loss, grad = cox.loss_grad(torch.from_numpy(beta).view(1, p).cuda())
    negL, g = oracle.loss_grad(M, d.time, d.event, beta.astype(np.float64))
    assert loss[0] == pytest.approx(negL, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(-grad.cpu().numpy()[0], g, rtol=0, atol=1e-6 * max(1e-30, np.abs(g).max()))


@pytest.mark.parametrize("storage,ldx", [("int8", 1003), ("int8", 1008), ("fp8", 1003), ("fp8", 1024)])
def test_ragged_shapes_geno(storage, ldx):
    d = coxsim.genotype_problem(1003, 41, 3, 0.3, 99, days=True)
    cox, M = device_problem(d, storage, ldx=ldx)
    beta = (0.2 * np.random.default_rng(1).standard_normal(41)).astype(np.float32)
    loss, grad = cox.loss_grad(torch.from_numpy(beta).view(1, -1).cuda())
    negL, g = oracle.loss_grad(M, d.time, d.event, beta.astype(np.float64))
    assert loss[0] == pytest.approx(negL, rel=1e-12)
    np.testing.assert_allclose(-grad.cpu().numpy()[0], g, rtol=0, atol=1e-6 * np.abs(g).max())


@pytest.mark.parametrize("storage,ldx", [("int8", 20011), ("fp8", 20016), ("f32", 20012), ("fp8", 20011)])
def test_row_splits(storage, ldx):
    # n spans several 8192-row splits of X' r, with a ragged tail
    d = coxsim.genotype_problem(20011, 70, 4, 0.3, 123, days=True)
    cox, M = device_problem(d, storage, ldx=ldx, max_batch=2)
    rng = np.random.default_rng(5)
    beta = (0.1 * rng.standard_normal((2, 70))).astype(np.float32)
    loss, grad = cox.loss_grad(torch.from_numpy(beta).cuda())
    for b in range(2):
        negL, g = oracle.loss_grad(M, d.time, d.event, beta[b].astype(np.float64))
        assert loss[b] == pytest.approx(negL, rel=1e-12)
        np.testing.assert_allclose(-grad.cpu().numpy()[b], g, rtol=0, atol=1e-6 * np.abs(g).max())
    lam = 0.3 * oracle.lambda_max(M, d.time, d.event)
    s2, _ = oracle.opnorm2(M)
    bo, tr, _, _ = oracle.fit(M, d.time, d.event, lam, 1 / (2 * s2), max_iter=25)
    bg, _, obj, _ = cox.fit_path([lam], max_iter=25, tol=0.0, step=1 / (2 * s2))
    assert rel_beta_err(bg.cpu().numpy()[0], bo) <= BETA_TOL
    assert obj[0] == pytest.approx(tr[-1], rel=OBJ_TOL)


@pytest.mark.parametrize("storage", ["f32", "int8", "fp8"])
def test_lambda_max_and_opnorm(c0, storage):
    cox, M = device_problem(c0, storage)
    lm = cox.lambda_max()
    assert lm == pytest.approx(oracle.lambda_max(M, c0.time, c0.event), rel=1e-6)
    s2, it = cox.opnorm2(tol=1e-10, maxiter=3000)
    s2o, _ = oracle.opnorm2(M, tol=1e-10, maxiter=3000)
    assert s2 == pytest.approx(s2o, rel=1e-6)
    assert s2 == pytest.approx(np.linalg.norm(M.to_dense64(), 2) ** 2, rel=1e-5)
    s2d, itd = cox.opnorm2()
    s2od, itod = oracle.opnorm2(M)
    assert s2d == pytest.approx(s2od, rel=1e-5)
    assert abs(itd - itod) <= 1


@pytest.mark.parametrize("storage", ["f32", "int8", "fp8"])
@pytest.mark.parametrize("eta_mode", [0, 1])
def test_fit_iterates_match_oracle(c0, storage, eta_mode):
    """The 1,000 x 2,000 oracle-sized problem: lambda = 0.5 lambda_max, 200 steps from beta = 0,
    compared at k = 1, 10, 100, 200."""
    cox, M = device_problem(c0, storage)
    lm = oracle.lambda_max(M, c0.time, c0.event)
    lam = 0.5 * lm
    sigma = _step(M, c0)
    for k in (1, 10, 100, 200):
        bo, tr, ko, _ = oracle.fit(M, c0.time, c0.event, lam, sigma, max_iter=k)
        beta, iters, obj, st = cox.fit_path([lam], max_iter=k, tol=0.0, step=sigma, eta_mode=eta_mode)
        assert iters[0] == k and st == P.ERR_NOT_CONVERGED
        assert rel_beta_err(beta.cpu().numpy()[0], bo) <= BETA_TOL, k
        assert obj[0] == pytest.approx(tr[-1], rel=OBJ_TOL)


def test_fit_gaussian_batch_and_groups():
    # B = 11 spans two VALU groups (8 + 3); each b must equal its own oracle run
    d = coxsim.gaussian_problem(1500, 300, 10, 0.3, 5)
    cox, M = device_problem(d, "f32", max_batch=11)
    lm = oracle.lambda_max(M, d.time, d.event)
    lams = coxsim.lambda_grid(lm, 11, 0.05)
    lams[0] *= 1 + 1e-6  # just above lambda_max: beta stays exactly zero
    sigma = _step(M, d)
    beta, iters, obj, st = cox.fit_path(lams, max_iter=60, tol=0.0, step=sigma)
    beta = beta.cpu().numpy()
    for b, lam in enumerate(lams):
        bo, tr, _, _ = oracle.fit(M, d.time, d.event, lam, sigma, max_iter=60)
        if np.abs(bo).max() > 0:
            assert rel_beta_err(beta[b], bo) <= BETA_TOL, b
        else:
            assert np.all(beta[b] == 0), b
        assert obj[b] == pytest.approx(tr[-1], rel=OBJ_TOL), b
    assert np.all(beta[0] == 0)


def test_convergence_rule_matches_oracle(c0):
    cox, M = device_problem(c0, "f32")
    lm = oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    for frac in (0.7, 0.4):
        bo, tr, ko, conv = oracle.fit(M, c0.time, c0.event, frac * lm, sigma, max_iter=3000, tol=1e-6, lag=10)
        beta, iters, obj, st = cox.fit_path([frac * lm], max_iter=3000, tol=1e-6, lag=10, step=sigma, poll=7)
        assert conv and st == P.OK
        assert abs(int(iters[0]) - ko) <= 1
        assert obj[0] == pytest.approx(tr[-1], rel=OBJ_TOL)
        if iters[0] == ko:
            assert rel_beta_err(beta.cpu().numpy()[0], bo) <= BETA_TOL


def test_default_step_is_paper_step(c0):
    cox, M = device_problem(c0, "f32")
    lam = 0.5 * oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    bo, tr, _, _ = oracle.fit(M, c0.time, c0.event, lam, sigma, max_iter=30)
    beta, _, obj, _ = cox.fit_path([lam], max_iter=30, tol=0.0, step=0.0)
    assert rel_beta_err(beta.cpu().numpy()[0], bo) <= BETA_TOL
    assert obj[0] == pytest.approx(tr[-1], rel=OBJ_TOL)


def test_prox_step_and_apply(c0):
    cox, M = device_problem(c0, "f32", max_batch=2)
    lm = oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    rng = np.random.default_rng(3)
    beta0 = (0.05 * rng.standard_normal((2, c0.p)) * (rng.random((2, c0.p)) < 0.1)).astype(np.float32)
    lams = np.array([0.5 * lm, 0.2 * lm])
    bt = torch.from_numpy(beta0.copy()).cuda()
    obj = cox.prox_step(bt, lams, sigma)
    got = bt.cpu().numpy()
    for b in range(2):
        bo, tr, _, _ = oracle.fit(M, c0.time, c0.event, lams[b], sigma, max_iter=1, beta0=beta0[b].astype(np.float64))
        assert rel_beta_err(got[b], bo) <= BETA_TOL
        assert obj[b] == pytest.approx(tr[0], rel=1e-12)
    # the standalone elementwise kernel: beta <- S_{sigma lam}(beta - sigma grad)
    bt2 = torch.from_numpy(beta0.copy()).cuda()
    _, grad = cox.loss_grad(bt2)
    cox.prox_apply(bt2, grad, lams, sigma)
    np.testing.assert_allclose(bt2.cpu().numpy(), got, rtol=0, atol=1e-6 * np.abs(got).max())


def test_warm_start_continues(c0):
    cox, M = device_problem(c0, "f32")
    lam = 0.4 * oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    b10, _, o10, _ = cox.fit_path([lam], max_iter=10, tol=0.0, step=sigma)
    b5, _, _, _ = cox.fit_path([lam], max_iter=5, tol=0.0, step=sigma)
    b5w, it, o5w, _ = cox.fit_path([lam], max_iter=5, tol=0.0, step=sigma, beta=b5.clone())
    assert rel_beta_err(b5w.cpu().numpy(), b10.cpu().numpy()) <= 1e-6
    assert o5w[0] == pytest.approx(o10[0], rel=1e-9)


def test_deterministic(c0):
    cox, M = device_problem(c0, "fp8")
    lam = 0.3 * oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    a, _, oa, _ = cox.fit_path([lam], max_iter=50, tol=0.0, step=sigma)
    a = a.clone()
    b, _, ob, _ = cox.fit_path([lam], max_iter=50, tol=0.0, step=sigma)
    assert torch.equal(a, b) and oa[0] == ob[0]


def test_no_events_and_degenerate():
    n, p = 300, 20
    d = coxsim.genotype_problem(n, p, 2, 0.3, 3)
    ev0 = np.zeros(n, np.int32)
    X = torch.from_numpy(d.standardized32()).cuda()
    cox = P.Cox(X, d.time, ev0)
    assert cox.lambda_max() == 0.0
    loss, grad = cox.loss_grad(torch.zeros((1, p), device="cuda"))
    assert loss[0] == 0.0 and torch.all(grad == 0)
    beta, iters, obj, st = cox.fit_path([0.1], max_iter=20, tol=1e-5, step=1e-3)
    assert torch.all(beta == 0) and obj[0] == 0.0 and iters[0] == 10 and st == P.OK
    # all subjects tied: every risk set is the whole sample
    tt = np.full(n, 5.0)
    cox2 = P.Cox(X, tt, d.event)
    bt = (0.1 * np.random.default_rng(0).standard_normal(p)).astype(np.float32)
    loss, grad = cox2.loss_grad(torch.from_numpy(bt).view(1, p).cuda())
    negL, g = oracle.loss_grad(oracle.Matrix.dense(d.standardized32()), tt, d.event, bt.astype(np.float64))
    assert loss[0] == pytest.approx(negL, rel=1e-12)
    np.testing.assert_allclose(-grad.cpu().numpy()[0], g, atol=1e-6 * np.abs(g).max())


def test_errors_through_the_abi(c0):
    cox, M = device_problem(c0, "f32", max_batch=2)
    with pytest.raises(P.CoxError) as e:
        cox.loss_grad(torch.zeros((3, c0.p), device="cuda"))
    assert e.value.status == P.ERR_INVALID_ARG
    bad = torch.zeros((1, c0.p), device="cuda")
    bad[0, 5] = float("nan")
    with pytest.raises(P.CoxError) as e:
        cox.loss_grad(bad)
    assert e.value.status == P.ERR_NUMERIC
    with pytest.raises(P.CoxError) as e:
        cox.fit_path([-1.0], max_iter=3)
    assert e.value.status == P.ERR_INVALID_ARG
    # the context still works after errors
    loss, _ = cox.loss_grad(torch.zeros((1, c0.p), device="cuda"))
    assert np.isfinite(loss[0])


def test_objective_trace(c0):
    """The per-step objective trace of cox_fit_path equals the oracle's f_0..f_K,
    step by step; a lambda that stops early has NaN past its last step."""
    cox, M = device_problem(c0, "fp8", max_batch=2)
    lm = oracle.lambda_max(M, c0.time, c0.event)
    sigma = _step(M, c0)
    lams = np.array([0.6 * lm, 1.5 * lm])  # the second stays at beta = 0 and meets the rule at k = lag
    beta, iters, obj, st, tr = cox.fit_path(lams, max_iter=60, tol=1e-9, lag=10, step=sigma, trace=True)
    assert tr.shape == (2, 61)
    bo, tro, ko, _ = oracle.fit(M, c0.time, c0.event, lams[0], sigma, max_iter=60, tol=1e-9, lag=10)
    assert iters[0] == ko
    np.testing.assert_allclose(tr[0, : ko + 1], tro, rtol=OBJ_TOL)
    assert np.all(np.isnan(tr[0, ko + 1:]))
    assert iters[1] == 10 and np.all(tr[1, :11] == tr[1, 0]) and np.all(np.isnan(tr[1, 11:]))
    assert tr[0, iters[0]] == obj[0] and tr[1, 10] == obj[1]


def test_fit_options_checked(c0):
    cox, M = device_problem(c0, "f32")
    L = P.lib()
    lam = np.array([0.5 * oracle.lambda_max(M, c0.time, c0.event)])
    beta = torch.zeros((1, c0.p), device="cuda")
    for field, bad in (("deterministic", 2), ("persistent", -1), ("eta_mode", 3), ("residual_bits", 8)):
        o = P.FitOpts(5, 0.0, 10, 1e-3, 0, 0, 1, 0, 16, 0, None)
        setattr(o, field, bad)
        st = L.cox_fit_path(cox._h, P._np_ptr(lam), 1, ctypes.byref(o), beta.data_ptr(), None, None)
        assert st == P.ERR_INVALID_ARG, field
    # deterministic = 0 and 1 run the same computation
    outs = []
    for det in (0, 1):
        o = P.FitOpts(5, 0.0, 10, 1e-3, 0, 0, det, 0, 16, 0, None)
        b = torch.zeros((1, c0.p), device="cuda")
        obj = np.zeros(1)
        st = L.cox_fit_path(cox._h, P._np_ptr(lam), 1, ctypes.byref(o), b.data_ptr(), None, P._np_ptr(obj))
        assert st == P.ERR_NOT_CONVERGED
        outs.append((b.cpu(), obj[0]))
    assert torch.equal(outs[0][0], outs[1][0]) and outs[0][1] == outs[1][1]
