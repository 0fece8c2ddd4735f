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
