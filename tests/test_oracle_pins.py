"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test ties the oracle to something other than itself: hand-derived closed
forms (tests/golden), an O(n^2) brute force built from the dense pi matrix of
Section 5.3, invariances of the partial likelihood, central finite
differences, a closed-form minimiser, an independent quasi-Newton solver, a
Newton MLE and an SVD.  A plausible slip in the oracle (a dropped term, a sign,
a wrong tie boundary, a transposed operand, lambda in place of sigma*lambda)
fails at least one of them.
"""
import math
import os

import numpy as np
import pytest
import scipy.optimize

import coxsim
import oracle
from tests import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "cox_closed_forms.txt")


def _golden_cases():
    cases = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        name, t, e, eta, L, r = [f.strip() for f in line.split("|")]
        ev = lambda s: [float(eval(x, {"math": math})) for x in s.split(",")]
        cases.append((name, ev(t), [int(x) for x in e.split(",")], ev(eta), ev(L)[0], ev(r)))
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c[0])
def test_closed_forms(case):
    _, t, e, eta, L_want, r_want = case
    L, r = oracle.loglik(eta, t, e)
    assert L == pytest.approx(L_want, rel=1e-14, abs=1e-15)
    np.testing.assert_allclose(r, r_want, rtol=1e-14, atol=1e-15)


def test_distinct_times_residual_formula():
    # distinct times, all events, eta = 0: the subject with the k-th smallest
    # time has c = sum_{i<=k} 1/(n-i+1) (harmonic tail), so r = 1 - c.
    n = 50
    t = np.random.default_rng(3).permutation(n).astype(float) + 1.0
    L, r = oracle.loglik(np.zeros(n), t, np.ones(n, np.int32))
    ranks = np.argsort(np.argsort(t))  # 0 = smallest time
    want = np.array([1.0 - sum(1.0 / (n - i) for i in range(k + 1)) for k in ranks])
    np.testing.assert_allclose(r, want, rtol=1e-13, atol=1e-14)
    assert L == pytest.approx(-math.lgamma(n + 1), rel=1e-13)


def _random_case(n, seed, ties=True, scale=1.0, censor=0.3):
    rng = np.random.default_rng(seed)
    t = rng.integers(1, max(2, n // 4), size=n).astype(float) if ties else rng.random(n)
    d = (rng.random(n) > censor).astype(np.int32)
    eta = scale * rng.standard_normal(n)
    return eta, t, d


@pytest.mark.parametrize("n,ties,scale", [(1, True, 1.0), (2, False, 1.0), (7, True, 1.0),
                                          (300, True, 2.0), (300, False, 3.0), (1500, True, 1.0),
                                          (400, True, 30.0)])
def test_scan_matches_bruteforce(n, ties, scale):
    eta, t, d = _random_case(n, 100 + n, ties, scale)
    L, r = oracle.loglik(eta, t, d)
    L_b = brute.loglik(eta, t, d)
    r_b = brute.residual(eta, t, d)
    assert L == pytest.approx(L_b, rel=1e-12, abs=1e-12)
    np.testing.assert_allclose(r, r_b, rtol=1e-10, atol=1e-12)


def test_invariants():
    eta, t, d = _random_case(500, 7, ties=True)
    L, r = oracle.loglik(eta, t, d)
    # sum r = 0: sum_k w_k c_k = sum_i delta_i
    assert abs(r.sum()) < 1e-11 * len(r)
    # shift invariance L(eta + c) = L(eta)
    L2, r2 = oracle.loglik(eta + 123.25, t, d)
    assert L2 == pytest.approx(L, rel=1e-12)
    np.testing.assert_allclose(r2, r, atol=1e-12)
    # strictly increasing transform of the times changes nothing
    L3, r3 = oracle.loglik(eta, np.exp(0.3 * t) + 5.0, d)
    assert L3 == pytest.approx(L, rel=1e-13)
    np.testing.assert_allclose(r3, r, atol=1e-13)
    # relabelling the subjects permutes r and leaves L alone (order within ties)
    perm = np.random.default_rng(1).permutation(len(t))
    L4, r4 = oracle.loglik(eta[perm], t[perm], d[perm])
    assert L4 == pytest.approx(L, rel=1e-12)
    np.testing.assert_allclose(r4, r[perm], atol=1e-12)
    # no events: L = 0 and r = 0
    L5, r5 = oracle.loglik(eta, t, np.zeros_like(d))
    assert L5 == 0.0 and np.all(r5 == 0.0)


def test_order_and_tie_groups():
    t = np.array([2.0, 5.0, 2.0, 1.0, 5.0, 5.0])
    o, gs, ge = oracle.order(t)
    np.testing.assert_array_equal(o, [1, 4, 5, 0, 2, 3])  # non-increasing, stable
    np.testing.assert_array_equal(gs, [0, 0, 0, 3, 3, 5])
    np.testing.assert_array_equal(ge, [2, 2, 2, 4, 4, 5])
    with pytest.raises(ValueError):
        oracle.order([1.0, float("nan")])


def _small_geno(n=200, p=12, seed=5, censor=0.3, k=3):
    d = coxsim.genotype_problem(n, p, k, censor, seed)
    X = oracle.Matrix.genotype(d.G, d.mu, d.s)
    return d, X


def test_xbeta_xtr_against_dense():
    d, X = _small_geno()
    Xd = X.to_dense64()
    beta = np.random.default_rng(2).standard_normal(X.p)
    r = np.random.default_rng(3).standard_normal(X.n)
    np.testing.assert_allclose(oracle.xbeta(X, beta), Xd.T @ beta, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(oracle.xtr(X, r), Xd @ r, rtol=1e-12, atol=1e-11)
    # the standardised columns have mean 0 and population variance 1
    np.testing.assert_allclose(Xd.mean(axis=1), 0.0, atol=1e-6)
    np.testing.assert_allclose((Xd ** 2).mean(axis=1), 1.0, rtol=1e-6)


def test_gradient_central_differences():
    d, X = _small_geno(n=300, p=8, seed=11)
    beta = 0.3 * np.random.default_rng(4).standard_normal(X.p)
    negL, g = oracle.loss_grad(X, d.time, d.event, beta)
    h = 1e-5
    fd = np.empty(X.p)
    for j in range(X.p):
        e = np.zeros(X.p)
        e[j] = h
        fp, _ = oracle.loss_grad(X, d.time, d.event, beta + e)
        fm, _ = oracle.loss_grad(X, d.time, d.event, beta - e)
        fd[j] = -(fp - fm) / (2 * h)  # dL/dbeta_j (loss is -L)
    np.testing.assert_allclose(g, fd, rtol=1e-7, atol=1e-7 * np.abs(g).max())
    assert negL == pytest.approx(-brute.loglik(X.to_dense64().T @ beta, d.time, d.event), rel=1e-12)
    np.testing.assert_allclose(g, brute.gradient(X.to_dense64(), beta, d.time, d.event), rtol=1e-9, atol=1e-9)


def test_soft_threshold_definition():
    st = oracle.soft_threshold
    assert st(3.0, 1.0) == 2.0 and st(-3.0, 1.0) == -2.0
    assert st(0.5, 1.0) == 0.0 and st(-0.5, 1.0) == 0.0
    assert st(1.0, 1.0) == 0.0 and st(-1.0, 1.0) == 0.0
    assert st(2.5, 0.0) == 2.5


@pytest.mark.parametrize("lam", [0.05, 0.2, 0.4, 0.5, 0.7])
def test_two_subject_minimiser(lam):
    # x = (1, 0), y = (1, 2), both events: -L(b) = -b + log(1 + e^b), whose
    # gradient is -1/(1+e^b), so lambda_max = 1/2 and the minimiser of
    # -L + lam |b| is log((1 - lam)/lam) for lam < 1/2, else 0.
    # ||X||_2^2 = 1, so the paper's step 1/(2 ||X||^2) is 1/2.
    X = oracle.Matrix.dense(np.array([[1.0, 0.0]]))
    t, e = [1.0, 2.0], [1, 1]
    assert oracle.lambda_max(X, t, e) == pytest.approx(0.5, rel=1e-15)
    s2, _ = oracle.opnorm2(X)
    assert s2 == pytest.approx(1.0, rel=1e-12)
    beta, trace, k, conv = oracle.fit(X, t, e, lam, 0.5, max_iter=20000, tol=0.0, lag=10)
    want = math.log((1 - lam) / lam) if lam < 0.5 else 0.0
    assert beta[0] == pytest.approx(want, rel=1e-9, abs=1e-12)
    assert trace[-1] == pytest.approx(-want + math.log1p(math.exp(want)) + lam * abs(want), rel=1e-12)


def test_lambda_max_boundary():
    d, X = _small_geno(n=400, p=30, seed=21)
    lm = oracle.lambda_max(X, d.time, d.event)
    _, g0 = oracle.loss_grad(X, d.time, d.event, np.zeros(X.p))
    # at beta = 0 every w_i = 1: c is the Nelson-Aalen cumulative hazard
    assert lm == pytest.approx(np.abs(brute.gradient(X.to_dense64(), np.zeros(X.p), d.time, d.event)).max(),
                               rel=1e-12)
    sigma = 1e-3
    b, _, _, _ = oracle.fit(X, d.time, d.event, lm * (1 + 1e-12), sigma, max_iter=1)
    assert np.all(b == 0.0)
    b, _, _, _ = oracle.fit(X, d.time, d.event, lm * (1 - 1e-3), sigma, max_iter=1)
    np.testing.assert_array_equal(np.nonzero(b)[0], [np.argmax(np.abs(g0))])
    # one step from zero is exactly S_{sigma lam}(sigma g0): threshold sigma*lam, not lam
    lam = 0.5 * lm
    b, _, _, _ = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=1)
    want = np.sign(g0) * np.maximum(np.abs(sigma * g0) - sigma * lam, 0.0)
    np.testing.assert_allclose(b, want, rtol=1e-14, atol=0)


def test_power_iteration_matches_svd():
    d, X = _small_geno(n=500, p=40, seed=31)
    s2, it = oracle.opnorm2(X, tol=1e-10, maxiter=5000)
    want = np.linalg.norm(X.to_dense64(), 2) ** 2
    assert s2 == pytest.approx(want, rel=1e-8)
    s2d, _ = oracle.opnorm2(X)  # the paper's defaults: tol 1e-6
    assert s2d == pytest.approx(want, rel=1e-4)
    Xg = oracle.Matrix.dense(np.random.default_rng(0).standard_normal((30, 200)).astype(np.float32))
    s2g, _ = oracle.opnorm2(Xg, tol=1e-12, maxiter=20000)
    assert s2g == pytest.approx(np.linalg.norm(Xg.to_dense64(), 2) ** 2, rel=1e-8)


def _bruteforce_optimum(Xd, y, delta, lam):
    """Minimise -L + lam ||beta||_1 with L-BFGS-B on beta = u - v, u, v >= 0,
    using the O(n^2) brute-force likelihood (independent of the oracle)."""
    p = Xd.shape[0]

    def fun(z):
        u, v = z[:p], z[p:]
        b = u - v
        g = brute.gradient(Xd, b, y, delta)
        f = -brute.loglik(Xd.T @ b, y, delta) + lam * z.sum()
        return f, np.concatenate([-g + lam, g + lam])

    res = scipy.optimize.minimize(fun, np.zeros(2 * p), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * (2 * p),
                                  options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12, maxcor=30))
    return res.x[:p] - res.x[p:], res.fun


@pytest.mark.parametrize("frac", [0.5, 0.2])
def test_ista_reaches_independent_optimum_and_kkt(frac):
    d, X = _small_geno(n=250, p=15, seed=41, k=4)
    Xd = X.to_dense64()
    lm = oracle.lambda_max(X, d.time, d.event)
    lam = frac * lm
    s2, _ = oracle.opnorm2(X)
    sigma = 1.0 / (2.0 * s2)
    beta, trace, k, conv = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=60000, tol=1e-16, lag=10)
    b_ref, f_ref = _bruteforce_optimum(Xd, d.time, d.event, lam)
    assert trace[-1] == pytest.approx(f_ref, rel=1e-9)
    assert trace[-1] <= f_ref + 1e-9 * abs(f_ref)
    # the paper's step 1/(2||X||^2) decreased the objective monotonically here
    assert np.all(np.diff(trace) <= 1e-12 * np.abs(trace[1:]))
    # KKT: |g_j| <= lam off the support, g_j = lam sign(beta_j) on it
    g = brute.gradient(Xd, beta, d.time, d.event)
    on = beta != 0
    assert on.any()
    assert np.all(np.abs(g[~on]) <= lam * (1 + 1e-6))
    np.testing.assert_allclose(g[on], lam * np.sign(beta[on]), rtol=1e-6)
    # prox-gradient residual is zero at the fixed point
    step = np.sign(beta + sigma * g) * np.maximum(np.abs(beta + sigma * g) - sigma * lam, 0.0)
    assert np.abs(beta - step).max() / sigma < 1e-6 * lam


def test_unpenalised_fit_matches_newton():
    # lambda = 0 and n >> p: ISTA must reach the Cox MLE, found here by Newton's
    # method on the brute-force likelihood.
    rng = np.random.default_rng(8)
    n, p = 400, 3
    Xd = rng.standard_normal((p, n))
    eta_true = Xd.T @ np.array([0.5, -0.3, 0.2])
    y, delta = coxsim.survival_times(eta_true, 0.3, rng)
    b = np.zeros(p)
    for _ in range(50):
        g = brute.gradient(Xd, b, y, delta)
        H = Xd @ brute.hessian_eta(Xd.T @ b, y, delta) @ Xd.T
        b = b + np.linalg.solve(H, g)
    X = oracle.Matrix.dense(Xd)
    s2, _ = oracle.opnorm2(X)
    beta, trace, k, conv = oracle.fit(X, y, delta, 0.0, 1.0 / (2 * s2), max_iter=20000, tol=1e-16)
    np.testing.assert_allclose(beta, b, rtol=1e-7, atol=1e-9)


def test_convergence_rule_and_trace():
    d, X = _small_geno(n=200, p=20, seed=51)
    lm = oracle.lambda_max(X, d.time, d.event)
    s2, _ = oracle.opnorm2(X)
    sigma = 1.0 / (2.0 * s2)
    beta, trace, k, conv = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=5000, tol=1e-5, lag=10)
    assert conv and k >= 10 and len(trace) == k + 1
    assert abs(trace[k] - trace[k - 10]) / (abs(trace[k]) + 1) < 1e-5
    assert all(abs(trace[j] - trace[j - 10]) / (abs(trace[j]) + 1) >= 1e-5 for j in range(10, k))
    # max_iter stops with the objective at beta_K recorded
    b5, tr5, k5, c5 = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=5)
    assert k5 == 5 and not c5 and len(tr5) == 6
    np.testing.assert_allclose(tr5, trace[:6], rtol=1e-15)
    f5 = brute.objective(X.to_dense64(), b5, d.time, d.event, 0.3 * lm)
    assert tr5[5] == pytest.approx(f5, rel=1e-12)
    # warm start continues the same sequence
    b10, _, _, _ = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=10)
    b10w, _, _, _ = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=5, beta0=b5)
    np.testing.assert_allclose(b10w, b10, rtol=1e-15, atol=0)


def test_iterate_history():
    """fit_history records each ISTA iterate: row k equals the result of k steps
    from zero, its trace is fit()'s, and each row is one proximal step (the
    soft threshold at sigma lambda of the brute-force gradient step) from the
    row before."""
    d, X = _small_geno(n=150, p=12, seed=53)
    lm = oracle.lambda_max(X, d.time, d.event)
    s2, _ = oracle.opnorm2(X)
    sigma, lam = 1.0 / (2.0 * s2), 0.4 * lm
    hist, trace, k = oracle.fit_history(X, d.time, d.event, lam, sigma, max_iter=7)
    assert k == 7 and hist.shape == (8, X.p) and not hist[0].any()
    _, tr, _, _ = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=7)
    np.testing.assert_array_equal(trace, tr)
    Xd = X.to_dense64()
    for j in range(1, 8):
        bj, _, _, _ = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=j)
        np.testing.assert_array_equal(hist[j], bj)
        g = brute.gradient(Xd, hist[j - 1], d.time, d.event)
        want = np.sign(hist[j - 1] + sigma * g) * np.maximum(np.abs(hist[j - 1] + sigma * g) - sigma * lam, 0.0)
        np.testing.assert_allclose(hist[j], want, rtol=1e-10, atol=1e-14)
