"""Iterate parity at the headline sizes, against the FP64 oracle, over many
steps.

The oracle cannot run ISTA over 200 GB, but ISTA's iterates stay sparse: a
column whose gradient never reaches the threshold is never moved.  The oracle
therefore runs on the columns that do move (regenerated from the counter hash),
and the GPU proves the restriction exact by evaluating the full gradient at
every oracle iterate (gpu_helpers.restricted_iterates).  What is checked:

* 400,000 x 500,000 FP8 genotypes, B = 64 lambdas from lambda_max to
  0.01 lambda_max, 25 batched steps from beta = 0 (matrix-core gradient and
  eta update): for lambdas whose support stays small, the GPU's iterate
  against the oracle's (1e-5 of max |beta|) and its objective -- evaluated
  from the eta the matrix-core update accumulated over 25 steps -- against
  the oracle's f at the same step (1e-6); the oracle's f and gradient at the
  GPU's own iterate; and, for all 64 lambdas, the accumulated objective
  against a fresh dense eta at the returned iterate, whose losses (three
  exact limb passes on the matrix cores) match the FP64 vector passes'
  (1e-13).
* 400,000 x 2,000, B = 64, 200 steps: iterates and objectives of three
  lambdas against the oracle's; the active-set eta update against a dense
  eta every step over the whole path.
* 200,000 x 200,000 FP8, lambda = 0.2 lambda_max, 60 steps: iterates and
  objective against the oracle's.
"""
import numpy as np
import pytest

import coxsim
import oracle
from tests.gpu_helpers import regenerate, rel_beta_err, restricted_iterates

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402


def _say(msg):
    print(f"[headline] {msg}", flush=True)


@pytest.fixture
def release():
    yield
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def _device(d, max_batch):
    ldx = (d.n + 15) // 16 * 16
    G, c1, c2 = coxsim.genotype_device(d.n, d.p, d.seed, d.thresholds, fmt=1, ldx=ldx)
    mu, s = coxsim.standardisation(c1, c2, d.n)
    cox = P.Cox(G, d.time, d.event, xtype=P.X_FP8_E4M3, n=d.n, center=torch.from_numpy(mu).cuda(),
                scale=torch.from_numpy(s).cuda(), max_batch=max_batch)
    return G, cox, mu, s


def test_batched_400k_x_500k_iterates_against_oracle(release, monkeypatch):
    d = coxsim.config4()
    _say("generating 400,000 x 500,000 FP8 genotypes")
    G, cox, mu, s = _device(d, 64)
    B, K = 64, 25
    lmax = cox.lambda_max()
    lams = coxsim.lambda_grid(lmax, B, 0.01)
    s2, _ = cox.opnorm2(maxiter=20)
    sigma = 1.0 / (2.0 * s2)
    beta, iters, obj, _ = cox.fit_path(lams, max_iter=K, tol=0.0, step=sigma)
    assert np.all(iters == K)
    assert cox.mfma_tuning()["xtr_variant"] >= 0 and cox.mfma_tuning()["eta_variant"] >= 0
    bh = beta.cpu().numpy().astype(np.float64)
    nnz = np.count_nonzero(bh, axis=1)
    _say(f"{K} steps done; nnz per lambda {nnz.min()}..{nnz.max()}")

    # every lambda: the objective from the accumulated eta against a dense eta at the returned iterate
    loss, _ = cox.loss_grad(beta, want_grad=False)
    f_dense = loss + lams * np.abs(bh).sum(axis=1)
    drift = np.abs(obj - f_dense) / np.abs(f_dense)
    _say(f"accumulated vs dense-eta objective over 64 lambdas: max rel. diff {drift.max():.2e}")
    assert drift.max() <= 1e-6
    # that dense eta ran as three exact limb passes on the matrix cores; the FP64 vector passes agree
    monkeypatch.setenv("COXHIP_NO_MFMA", "1")
    loss_v, _ = cox.loss_grad(beta, want_grad=False)
    monkeypatch.delenv("COXHIP_NO_MFMA")
    dense_rel = np.abs(loss - loss_v) / np.abs(loss_v)
    _say(f"dense eta, matrix-core limb passes vs FP64 vector passes: max rel. loss diff {dense_rel.max():.2e}")
    assert dense_rel.max() <= 1e-13

    # lambda_0 = lambda_max puts the leading column exactly at its threshold (a tie decided by rounding);
    # the lambdas below it have well-separated supports
    small = [b for b in range(1, B) if 0 < nnz[b] <= 2500]
    assert len(small) >= 3, nnz
    picks = [small[0], small[len(small) // 2], small[-1]]
    rng = np.random.default_rng(11)
    for b in picks:
        lam = lams[b]
        _, g_gpu_all = cox.loss_grad(beta[b : b + 1].contiguous())
        g_gpu = -g_gpu_all.cpu().numpy()[0].astype(np.float64)
        cand = np.union1d(np.flatnonzero(bh[b]), np.flatnonzero(np.abs(g_gpu) > 0.8 * lam))
        cols, hist, trace = restricted_iterates(cox, d, mu, s, lam, sigma, K, cand, say=_say)
        assert np.all(np.isin(np.flatnonzero(bh[b]), cols))
        e = rel_beta_err(bh[b, cols], hist[K])
        ef = abs(obj[b] - trace[K]) / abs(trace[K])
        # the oracle at the GPU's own iterate: f and the gradient on the support plus 48 sampled columns
        chk = np.union1d(np.flatnonzero(bh[b]), rng.choice(d.p, 48, replace=False))
        M = regenerate(d, mu, s, chk)
        eta = oracle.xbeta(M, bh[b, chk])
        L, r = oracle.loglik(eta, d.time, d.event)
        f_at = -L + lam * np.abs(bh[b]).sum()
        g_or = oracle.xtr(M, r)
        eg = np.abs(g_gpu[chk] - g_or).max() / np.abs(g_or).max()
        _say(f"lambda_{b} = {lam:.6g}: |S| = {nnz[b]}, oracle on {cols.size} columns; beta rel. err {e:.2e}, "
             f"objective rel. diff {ef:.2e} (oracle f at the GPU's beta: {abs(obj[b] - f_at) / abs(f_at):.2e}), "
             f"gradient rel. err {eg:.2e}")
        assert e <= 1e-5, (b, e)
        assert ef <= 1e-6, (b, ef)
        assert abs(obj[b] - f_at) <= 1e-6 * abs(f_at), b
        assert eg <= 1e-6, (b, eg)
    del G


def test_batched_long_run_at_n_400k(release):
    """200 batched steps at the real n over a change list that covers most of
    the 2,000 columns: the matrix-core eta update accumulated over the whole
    run against the oracle, and against a dense eta every step."""
    d = coxsim.genotype_problem(400000, 2000, 40, 0.80, 4712)
    G, cox, mu, s = _device(d, 64)
    B, K = 64, 200
    M = oracle.Matrix.genotype(d.G, d.mu, d.s)
    lams = coxsim.lambda_grid(oracle.lambda_max(M, d.time, d.event), B, 0.01)
    lams[0] *= 1 + 1e-6
    sigma = 1.0 / (2.0 * cox.opnorm2()[0])
    beta, _, obj, _ = cox.fit_path(lams, max_iter=K, tol=0.0, step=sigma)
    beta_d, _, obj_d, _ = cox.fit_path(lams, max_iter=K, tol=0.0, step=sigma, eta_mode=1)
    b_up, b_dn = beta.cpu().numpy(), beta_d.cpu().numpy()
    scale = np.abs(b_dn).max(axis=1)
    worst_mode = max(np.abs(b_up[b] - b_dn[b]).max() / scale[b] for b in range(1, B))
    worst_fmode = (np.abs(obj - obj_d) / np.abs(obj_d)).max()
    _say(f"{K} steps: active-set vs dense eta: beta {worst_mode:.2e}, objective {worst_fmode:.2e}; "
         f"nnz up to {np.count_nonzero(b_up, axis=1).max()} of {d.p}")
    assert worst_mode <= 1e-5 and worst_fmode <= 1e-6
    worst = 0.0
    for b in (3, 31, 63):
        bo, tr, _, _ = oracle.fit(M, d.time, d.event, lams[b], sigma, max_iter=K)
        e = rel_beta_err(b_up[b], bo)
        ef = abs(obj[b] - tr[-1]) / abs(tr[-1])
        worst = max(worst, e)
        _say(f"lambda_{b}: beta rel. err {e:.2e}, objective rel. diff {ef:.2e}, nnz {np.count_nonzero(bo)}")
        assert e <= 1e-5, (b, e)
        assert ef <= 1e-6, (b, ef)
    del G


def test_fp8_200k_x_200k_iterates_against_oracle(release):
    d = coxsim.config3()
    G, cox, mu, s = _device(d, 64)
    K = 60
    lam = 0.2 * cox.lambda_max()
    s2, _ = cox.opnorm2()
    sigma = 1.0 / (2.0 * s2)
    beta, _, obj, _ = cox.fit_path([lam], max_iter=K, tol=0.0, step=sigma)
    b = beta.cpu().numpy()[0].astype(np.float64)
    _, g = cox.loss_grad(beta)
    g = -g.cpu().numpy()[0].astype(np.float64)
    cand = np.union1d(np.flatnonzero(b), np.flatnonzero(np.abs(g) > 0.8 * lam))
    cols, hist, trace = restricted_iterates(cox, d, mu, s, lam, sigma, K, cand, say=_say)
    e = rel_beta_err(b[cols], hist[K])
    ef = abs(obj[0] - trace[K]) / abs(trace[K])
    _say(f"200,000 x 200,000 FP8, {K} steps: |S| = {np.count_nonzero(b)}, oracle on {cols.size} columns; "
         f"beta rel. err {e:.2e}, objective rel. diff {ef:.2e}")
    assert np.all(np.isin(np.flatnonzero(b), cols))
    assert e <= 1e-5
    assert ef <= 1e-6
    del G
