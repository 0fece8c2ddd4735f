"""GPU parity of the covariate block and the penalty factors (Section 6's
application: sex and the top principal components enter the model unpenalised
beside the SNPs), through the C ABI, against the FP64 oracle run on the dense
matrix [X~ | Z] with the same penalty factors.

Tolerances as for the plain path: relative objective <= 1e-6 and
max|beta - beta_oracle| <= 1e-5 max|beta_oracle| at the same step from the same
start; gradients to 1e-6 of their largest entry; lambda_max (whose covariate
sub-problem the GPU solves by ISTA to a gradient 1e-10 of its start and the
oracle by Newton) to 1e-6 relative.
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
Q = 11  # sex and ten principal components


@pytest.fixture(scope="module")
def prob():
    # ragged n (not a multiple of the 8192-row covariate blocks or of 256), tied days
    d, Z, gamma = coxsim.genotype_problem_with_covariates(3001, 700, 12, Q, 0.8, 9090, days=True)
    return d, Z


def _setup(prob, storage, B, ldz=None):
    d, Z = prob
    ldx = (d.n + 15) // 16 * 16
    cox, M = device_problem(d, storage, ldx=ldx, max_batch=B)
    ldz = d.n if ldz is None else ldz
    Zd = torch.zeros((Q, ldz), dtype=torch.float32)
    Zd[:, : d.n] = torch.from_numpy(Z)
    Zd = Zd.cuda()
    cox.set_covariates(Zd)
    Mo = oracle.Matrix.dense(np.vstack([M.to_dense64(), Z.astype(np.float64)]))
    return cox, Mo


def _factors(p, rng, zeros=0):
    pf = np.concatenate([rng.choice([0.5, 1.0, 2.0], size=p), np.zeros(Q)])
    if zeros:
        pf[rng.choice(p, zeros, replace=False)] = 0.0
    return pf


@pytest.mark.parametrize("storage,B", [("f32", 1), ("int8", 1), ("fp8", 5), ("fp8", 64), ("int8", 20)])
def test_fit_with_covariates_and_penalty_factors(prob, storage, B):
    d, Z = prob
    cox, Mo = _setup(prob, storage, B)
    rng = np.random.default_rng(B)
    pf = _factors(d.p, rng, zeros=3)  # three SNPs unpenalised as well
    cox.set_penalty_factors(pf)
    lm, _ = oracle.lambda_max_pf(Mo, d.time, d.event, np.where(pf > 0, pf, 0.0))
    lams = coxsim.lambda_grid(lm, B, 0.05) if B > 1 else np.array([0.3 * lm])
    sigma = 1.0 / (2.0 * oracle.opnorm2(Mo)[0])
    K = 25
    beta, _, obj, _ = cox.fit_path(lams, max_iter=K, tol=0.0, step=sigma)
    beta = beta.cpu().numpy()
    assert beta.shape == (B, d.p + Q)
    worst = 0.0
    for b in sorted({0, B // 2, B - 1}):
        bo, tr, _, _ = oracle.fit(Mo, d.time, d.event, lams[b], sigma, max_iter=K, pf=pf)
        e = rel_beta_err(beta[b], bo)
        worst = max(worst, e)
        assert e <= BETA_TOL, (b, e)
        assert obj[b] == pytest.approx(tr[-1], rel=OBJ_TOL), b
        assert np.all(bo[-Q:] != 0)  # the unpenalised covariates moved
    print(f"worst relative beta error with covariates and penalty factors: {worst:.2e}")


def test_lambda_max_with_free_covariates(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "fp8", 1)
    rng = np.random.default_rng(3)
    pf = _factors(d.p, rng)
    cox.set_penalty_factors(pf)
    want, _ = oracle.lambda_max_pf(Mo, d.time, d.event, pf)
    got = cox.lambda_max()
    assert got == pytest.approx(want, rel=1e-6)
    # penalised covariates stay at zero in the sub-problem
    pf2 = pf.copy()
    pf2[d.p + 3] = 1.5
    cox.set_penalty_factors(pf2)
    want2, _ = oracle.lambda_max_pf(Mo, d.time, d.event, pf2)
    assert cox.lambda_max() == pytest.approx(want2, rel=1e-6)
    # an unpenalised SNP is not served here
    pf3 = pf.copy()
    pf3[5] = 0.0
    cox.set_penalty_factors(pf3)
    with pytest.raises(P.CoxError) as ei:
        cox.lambda_max()
    assert ei.value.status == P.ERR_UNSUPPORTED
    # every column penalised: the closed form at beta = 0 (the gradient of X's
    # columns comes from the FP32 residual, as in the plain lambda_max)
    pf4 = np.where(pf > 0, pf, 1.0)
    cox.set_penalty_factors(pf4)
    want4, _ = oracle.lambda_max_pf(Mo, d.time, d.event, pf4)
    assert cox.lambda_max() == pytest.approx(want4, rel=1e-6)


@pytest.mark.parametrize("storage,B", [("f32", 3), ("int8", 16)])
def test_loss_grad_with_covariates(prob, storage, B):
    d, Z = prob
    cox, Mo = _setup(prob, storage, B)
    rng = np.random.default_rng(9)
    beta = (0.05 * rng.standard_normal((B, d.p + Q)) * (rng.random((B, d.p + Q)) < 0.3)).astype(np.float32)
    loss, grad = cox.loss_grad(torch.from_numpy(beta).cuda())
    grad = grad.cpu().numpy()
    assert grad.shape == (B, d.p + Q)
    for b in range(B):
        negL, g = oracle.loss_grad(Mo, d.time, d.event, beta[b].astype(np.float64))
        assert loss[b] == pytest.approx(negL, rel=1e-12)
        assert np.abs(grad[b] + g).max() <= 1e-6 * np.abs(g).max(), b


def test_opnorm2_with_covariates(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "int8", 1)
    s2, it = cox.opnorm2(tol=1e-10, maxiter=5000)
    want = np.linalg.norm(Mo.to_dense64(), 2) ** 2
    assert s2 == pytest.approx(want, rel=1e-7)
    s2d, itd = cox.opnorm2()
    so, ito = oracle.opnorm2(Mo)
    assert s2d == pytest.approx(so, rel=1e-6)


def test_prox_step_and_apply_with_penalty_factors(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "fp8", 4)
    rng = np.random.default_rng(4)
    pf = _factors(d.p, rng, zeros=2)
    cox.set_penalty_factors(pf)
    lm, _ = oracle.lambda_max_pf(Mo, d.time, d.event, pf * (pf > 0))
    lams = np.array([0.9, 0.5, 0.2, 0.05]) * lm
    sigma = 1.0 / (2.0 * oracle.opnorm2(Mo)[0])
    b0 = (0.03 * rng.standard_normal((4, d.p + Q)) * (rng.random((4, d.p + Q)) < 0.2)).astype(np.float32)
    beta = torch.from_numpy(b0).cuda()
    obj = cox.prox_step(beta, lams, sigma)
    got = beta.cpu().numpy()
    for b in range(4):
        bo, tr, _, _ = oracle.fit(Mo, d.time, d.event, lams[b], sigma, max_iter=1, beta0=b0[b], pf=pf)
        assert obj[b] == pytest.approx(tr[0], rel=1e-10)
        assert rel_beta_err(got[b], bo) <= BETA_TOL
    # the elementwise kernel alone, with the same factors
    gr = (0.5 * rng.standard_normal((4, d.p + Q))).astype(np.float32)
    bt = torch.from_numpy(b0).cuda()
    cox.prox_apply(bt, torch.from_numpy(gr).cuda(), lams, sigma)
    x = b0.astype(np.float64) - sigma * gr.astype(np.float64)
    t = sigma * lams[:, None] * pf[None, :]
    want = np.sign(x) * np.maximum(np.abs(x) - t, 0.0)
    np.testing.assert_allclose(bt.cpu().numpy(), want.astype(np.float32), rtol=1e-6, atol=1e-12)


def test_fit_sequence_is_the_warm_started_oracle(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "int8", 1)
    lm = cox.lambda_max()
    lams = lm * np.array([0.8, 0.5, 0.3, 0.15])
    sigma = 1.0 / (2.0 * oracle.opnorm2(Mo)[0])
    pf = np.concatenate([np.ones(d.p), np.zeros(Q)])
    K = 15
    path, iters, obj, st = cox.fit_sequence(lams, max_iter=K, tol=0.0, step=sigma)
    assert st == P.ERR_NOT_CONVERGED and np.all(iters == K)
    path = path.cpu().numpy()
    bo = np.zeros(d.p + Q)
    for l, lam in enumerate(lams):
        # the GPU hands each solution on in FP32
        bo, tr, _, _ = oracle.fit(Mo, d.time, d.event, lam, sigma, max_iter=K, beta0=bo.astype(np.float32), pf=pf)
        assert rel_beta_err(path[l], bo) <= BETA_TOL, l
        assert obj[l] == pytest.approx(tr[-1], rel=OBJ_TOL), l
    # with the paper's rule (lag 10, 1e-5) every lambda stops by itself
    path2, iters2, obj2, st2 = cox.fit_sequence(lams, max_iter=5000, tol=1e-5, lag=10, step=sigma)
    assert st2 == P.OK and np.all(iters2 >= 10) and np.all(iters2 < 5000)


def test_removing_covariates_restores_the_plain_path(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "int8", 1)
    cox.set_covariates(None)
    assert cox.ptot == d.p
    cox0, M = device_problem(d, "int8", ldx=(d.n + 15) // 16 * 16)
    lm = cox0.lambda_max()
    assert cox.lambda_max() == lm
    sigma = 1.0 / (2.0 * oracle.opnorm2(M)[0])
    a, _, oa, _ = cox.fit_path([0.3 * lm], max_iter=10, tol=0.0, step=sigma)
    b, _, ob, _ = cox0.fit_path([0.3 * lm], max_iter=10, tol=0.0, step=sigma)
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    np.testing.assert_array_equal(oa, ob)


def test_covariate_argument_checks(prob):
    d, Z = prob
    cox, Mo = _setup(prob, "f32", 1)
    with pytest.raises(P.CoxError) as ei:
        cox.set_penalty_factors(np.full(d.p + Q, -1.0))
    assert ei.value.status == P.ERR_INVALID_ARG
    short = torch.zeros((Q, d.n - 1), dtype=torch.float32, device="cuda")
    with pytest.raises(P.CoxError) as ei:
        cox.set_covariates(short)
    assert ei.value.status == P.ERR_INVALID_ARG
    big = torch.zeros((P.MAX_COVARIATES + 1, d.n), dtype=torch.float32, device="cuda")
    with pytest.raises(P.CoxError):
        cox.set_covariates(big)


@pytest.mark.parametrize("storage,B", [("int8", 6), ("fp8", 40)])
def test_early_stopping_lambdas_with_covariates(prob, storage, B):
    """Lambdas that meet the lag-10 rule at different steps stop while the rest
    go on: each one's steps, objective and beta match the oracle's own run
    under the same rule (the covariate block must leave a stopped lambda
    untouched)."""
    d, Z = prob
    cox, Mo = _setup(prob, storage, B)
    pf = np.concatenate([np.ones(d.p), np.zeros(Q)])
    lm, _ = oracle.lambda_max_pf(Mo, d.time, d.event, pf)
    lams = coxsim.lambda_grid(lm, B, 0.05)
    sigma = 1.0 / (2.0 * oracle.opnorm2(Mo)[0])
    beta, iters, obj, st = cox.fit_path(lams, max_iter=400, tol=1e-6, lag=10, step=sigma)
    beta = beta.cpu().numpy()
    assert len(set(iters.tolist())) > 1  # they did stop at different steps
    for b in sorted({0, B // 3, B - 1}):
        bo, tr, k, conv = oracle.fit(Mo, d.time, d.event, lams[b], sigma, max_iter=400, tol=1e-6, lag=10, pf=pf)
        assert abs(int(iters[b]) - k) <= 1, (b, iters[b], k)
        if int(iters[b]) == k:
            assert rel_beta_err(beta[b], bo) <= BETA_TOL, b
            assert obj[b] == pytest.approx(tr[-1], rel=OBJ_TOL), b
