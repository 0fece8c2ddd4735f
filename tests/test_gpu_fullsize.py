"""Parity at the full sizes of the two genotype workloads, on sampled outputs
the oracle can compute one by one.

At beta = 0 every weight is 1, so r(0) depends only on the times and events,
and g_j(0) = x~_j' r(0) needs only column j: the oracle regenerates sampled
columns from the counter hash and evaluates them.  One ISTA step from zero
gives beta_1j = S_{sigma lambda}(sigma g_j(0)) column by column, which checks
the batched matrix-core pass (quantised residual, int32 accumulation, proximal
epilogue) for all 64 lambdas at 400,000 x 500,000.
"""
import numpy as np
import pytest

import coxsim
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402


def _device_problem(d, fmt=1):
    ldx = (d.n + 15) // 16 * 16
    G, c1, c2 = coxsim.genotype_device(d.n, d.p, d.seed, d.thresholds, fmt=fmt, ldx=ldx)
    mu, s = coxsim.standardisation(c1, c2, d.n)
    return G, mu, s


def _oracle_g0(d, mu, s, cols):
    Gh = coxsim.genotype_columns(d.n, cols, d.seed, d.thresholds[cols])
    M = oracle.Matrix.genotype(Gh, mu[cols], s[cols])
    _, r0 = oracle.loglik(np.zeros(d.n), d.time, d.event)
    return oracle.xtr(M, r0), Gh


@pytest.fixture
def release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def test_fp8_200k_gradient_at_zero(release):
    d = coxsim.config3()
    G, mu, s = _device_problem(d, fmt=1)
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=d.n, center=torch.from_numpy(mu).cuda(),
                scale=torch.from_numpy(s).cuda())
    _, grad = cox.loss_grad(torch.zeros((1, d.p), device="cuda"))
    cols = np.sort(np.random.default_rng(1).choice(d.p, 48, replace=False))
    go, Gh = _oracle_g0(d, mu, s, cols)
    # the device generator wrote the same allele counts as the host twin
    codes = G[torch.from_numpy(cols).cuda(), : d.n].cpu().numpy()
    np.testing.assert_array_equal(codes, coxsim.FP8_E4M3_CODE[Gh])
    got = -grad.cpu().numpy()[0, cols].astype(np.float64)
    assert np.abs(got - go).max() <= 1e-6 * np.abs(go).max()
    lm = cox.lambda_max()
    assert lm >= np.abs(go).max() * (1 - 1e-6)


def test_batched_400k_x_500k_first_step(release):
    d = coxsim.config4()
    G, mu, s = _device_problem(d, fmt=1)
    B = 64
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=d.n, center=torch.from_numpy(mu).cuda(),
                scale=torch.from_numpy(s).cuda(), max_batch=B)
    cols = np.sort(np.random.default_rng(2).choice(d.p, 48, replace=False))
    go, _ = _oracle_g0(d, mu, s, cols)
    lmax = cox.lambda_max()
    lams = coxsim.lambda_grid(lmax, B, 0.01)
    sigma = 1e-7
    beta0, it0, f0, _ = cox.fit_path(lams, max_iter=0, tol=0.0, step=sigma)
    beta1, it1, f1, _ = cox.fit_path(lams, max_iter=1, tol=0.0, step=sigma)
    assert np.all(it1 == 1) and np.all(it0 == 0)
    b1 = beta1.cpu().numpy()[:, cols].astype(np.float64)
    want = np.sign(go)[None, :] * np.maximum(np.abs(sigma * go)[None, :] - sigma * lams[:, None], 0.0)
    scale = np.abs(want).max()
    assert scale > 0
    assert np.abs(b1 - want).max() <= 1e-5 * scale
    # zero exactly where |g_j(0)| <= lambda_b (away from ties with the threshold)
    clear = np.abs(np.abs(go)[None, :] - lams[:, None]) > 1e-6 * lams[:, None]
    assert np.all(((b1 == 0) == (want == 0))[clear])
    # the objective decreased for every lambda
    assert np.all(f1 <= f0)
    assert np.allclose(f0, f0[0], rtol=1e-12)


def test_fp32_gaussian_20k_x_50k_iterates(release):
    """The plain FP32 method at its full size (20,000 x 50,000 Gaussian X,
    lambda = 0.3 lambda_max, the power-iteration step): GPU and FP64 oracle
    iterates after 20 steps from beta = 0, element by element."""
    d = coxsim.config1()
    X = torch.from_numpy(d.X32).cuda()
    cox = P.Cox(X, d.time, d.event)
    M = oracle.Matrix.dense(d.X32)
    lam = 0.3 * oracle.lambda_max(M, d.time, d.event)
    s2, _ = cox.opnorm2()
    sigma = 1.0 / (2.0 * s2)
    K = 20
    beta, _, obj, _ = cox.fit_path([lam], max_iter=K, tol=0.0, step=sigma)
    bo, tr, _, _ = oracle.fit(M, d.time, d.event, lam, sigma, max_iter=K)
    b = beta.cpu().numpy()[0].astype(np.float64)
    rel = np.abs(b - bo).max() / np.abs(bo).max()
    print(f"\nFP32 20,000 x 50,000 after {K} steps: max|beta - beta_oracle| / max|beta_oracle| = {rel:.2e}, "
          f"objective rel. diff {abs(obj[0] - tr[-1]) / abs(tr[-1]):.2e}, nnz {np.count_nonzero(bo)}")
    assert rel <= 1e-5
    assert obj[0] == pytest.approx(tr[-1], rel=1e-6)


def test_batched_iterates_at_n_400k(release):
    """The batched matrix-core path at the real n: 400,000 x 2,000 FP8
    genotypes (same generator), 64 lambdas from lambda_max to 0.01 lambda_max,
    10 steps from beta = 0; GPU iterates against the FP64 oracle's at three
    lambdas across the path."""
    d = coxsim.genotype_problem(400000, 2000, 40, 0.80, 4711)
    G, mu, s = _device_problem(d, fmt=1)
    B = 64
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=d.n, center=torch.from_numpy(mu).cuda(),
                scale=torch.from_numpy(s).cuda(), max_batch=B)
    M = oracle.Matrix.genotype(d.G, d.mu, d.s)
    lams = coxsim.lambda_grid(oracle.lambda_max(M, d.time, d.event), B, 0.01)
    lams[0] *= 1 + 1e-6
    sigma = 1.0 / (2.0 * cox.opnorm2()[0])  # an input to both sides
    K = 10
    beta, _, obj, _ = cox.fit_path(lams, max_iter=K, tol=0.0, step=sigma)
    beta = beta.cpu().numpy()
    assert cox.mfma_tuning()["xtr_variant"] >= 0  # the matrix-core pass ran
    worst = 0.0
    for b in (5, 32, 63):
        bo, tr, _, _ = oracle.fit(M, d.time, d.event, lams[b], sigma, max_iter=K)
        e = np.abs(beta[b] - bo).max() / np.abs(bo).max()
        worst = max(worst, e)
        assert e <= 1e-5, (b, e)
        assert obj[b] == pytest.approx(tr[-1], rel=1e-6), b
    print(f"\nbatched FP8 400,000 x 2,000, B = 64, {K} steps: worst max|beta - beta_oracle| / max|beta_oracle| "
          f"over sampled lambdas = {worst:.2e}")
