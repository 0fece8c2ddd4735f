"""Pins of the oracle's penalty factors, its unpenalised Newton fit and its
lambda_max with unpenalised columns (Section 6's application: sex and the top
principal components enter the model without penalty).

What pins them, other than the oracle itself:
  * pf = 1 everywhere reproduces the plain l1 fit bit for bit;
  * an independent L-BFGS-B solve of the weighted problem on the O(n^2)
    brute-force likelihood, and the weighted KKT conditions;
  * the Newton fit against the brute-force gradient (zero at the result) and
    its inverse information against a central finite-difference Hessian of the
    brute-force gradient;
  * lambda_max against a brute-force sub-problem solve, and its defining
    property: just above it every penalised coefficient stays at zero, just
    below it the column that attains it enters.
"""
import numpy as np
import pytest
import scipy.optimize

import coxsim
import oracle
from tests import brute


def _problem(n=300, p=14, q=4, seed=61, days=True):
    d, Z, gamma = coxsim.genotype_problem_with_covariates(n, p, 3, q, 0.3, seed, days=days)
    G = oracle.Matrix.genotype(d.G, d.mu, d.s).to_dense64()
    Xd = np.vstack([G, Z.astype(np.float64)])
    return d, Xd, oracle.Matrix.dense(Xd)


def _weights(p, q, rng):
    pf = np.concatenate([rng.choice([0.5, 1.0, 2.0], size=p), np.zeros(q)])
    return pf


def test_unit_penalty_factors_are_the_plain_fit():
    d, Xd, X = _problem()
    lm = oracle.lambda_max(X, d.time, d.event)
    sigma = 1.0 / (2.0 * oracle.opnorm2(X)[0])
    a, ta, ka, _ = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=200)
    b, tb, kb, _ = oracle.fit(X, d.time, d.event, 0.3 * lm, sigma, max_iter=200, pf=np.ones(X.p))
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ta, tb)


def _weighted_bruteforce_optimum(Xd, y, delta, lam, pf):
    """min -L + lam sum_j pf_j |beta_j| with L-BFGS-B on beta = u - v, u, v >= 0."""
    p = Xd.shape[0]

    def fun(z):
        u, v = z[:p], z[p:]
        b = u - v
        g = brute.gradient(Xd, b, y, delta)
        f = -brute.loglik(Xd.T @ b, y, delta) + lam * (pf * (u + v)).sum()
        return f, np.concatenate([-g + lam * pf, g + lam * pf])

    res = scipy.optimize.minimize(fun, np.zeros(2 * p), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * (2 * p),
                                  options=dict(maxiter=50000, ftol=1e-16, gtol=1e-12, maxcor=30))
    return res.x[:p] - res.x[p:], res.fun


def test_weighted_fit_reaches_independent_optimum_and_kkt():
    d, Xd, X = _problem(n=250, p=12, q=3, seed=62)
    pf = _weights(12, 3, np.random.default_rng(3))
    lm, _ = oracle.lambda_max_pf(X, d.time, d.event, pf)
    lam = 0.3 * lm
    sigma = 1.0 / (2.0 * oracle.opnorm2(X)[0])
    beta, trace, k, conv = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=200000, tol=1e-16, pf=pf)
    b_ref, f_ref = _weighted_bruteforce_optimum(Xd, d.time, d.event, lam, pf)
    f_brute = brute.objective(Xd, beta, d.time, d.event, 0.0) + lam * (pf * np.abs(beta)).sum()
    assert trace[-1] == pytest.approx(f_brute, rel=1e-12)
    assert trace[-1] == pytest.approx(f_ref, rel=1e-9)
    g = brute.gradient(Xd, beta, d.time, d.event)
    free = pf == 0
    on = (beta != 0) & ~free
    off = (beta == 0) & ~free
    assert on.any() and off.any()
    assert np.abs(g[free]).max() <= 1e-6 * lam            # unpenalised: gradient zero
    assert np.all(np.abs(g[off]) <= lam * pf[off] * (1 + 1e-6))
    np.testing.assert_allclose(g[on], lam * pf[on] * np.sign(beta[on]), rtol=1e-6)
    # a threshold of sigma*lam*pf_j, not sigma*lam: one step from zero
    b1, _, _, _ = oracle.fit(X, d.time, d.event, lam, sigma, max_iter=1, pf=pf)
    g0 = brute.gradient(Xd, np.zeros(X.p), d.time, d.event)
    want = np.sign(g0) * np.maximum(np.abs(sigma * g0) - sigma * lam * pf, 0.0)
    np.testing.assert_allclose(b1, want, rtol=1e-13, atol=1e-300)


def test_newton_against_bruteforce_gradient_and_hessian():
    d, Xd, X = _problem(n=240, p=10, q=3, seed=63)
    cols = np.array([1, 4, 10, 11, 12])          # two SNPs and the three covariates
    fixed = np.zeros(X.p)
    fixed[7] = 0.4                               # another coefficient held fixed, not zero
    b, cov, it, conv = oracle.newton(X, d.time, d.event, cols, beta_fixed=fixed, gtol=1e-11)
    assert conv and it >= 2
    full = fixed.copy()
    full[cols] = b
    g = brute.gradient(Xd, full, d.time, d.event)
    assert np.abs(g[cols]).max() <= 1e-9
    # -Hessian by central differences of the brute-force gradient
    h = 1e-5
    H = np.empty((cols.size, cols.size))
    for a, j in enumerate(cols):
        e = np.zeros(X.p)
        e[j] = h
        H[:, a] = -(brute.gradient(Xd, full + e, d.time, d.event)[cols] -
                    brute.gradient(Xd, full - e, d.time, d.event)[cols]) / (2 * h)
    np.testing.assert_allclose(np.linalg.inv(cov), H, rtol=1e-6, atol=1e-6 * np.abs(H).max())
    # the same inverse information from the brute-force eta-space Hessian
    Hb = Xd[cols] @ brute.hessian_eta(Xd.T @ full, d.time, d.event) @ Xd[cols].T
    np.testing.assert_allclose(cov, np.linalg.inv(Hb), rtol=1e-9)


def test_newton_matches_three_subject_closed_form():
    # x = (1, 0, 1), times (1, 2, 3), events (1, 1, 0).  Risk sets {0, 1, 2} and
    # {1, 2}: L(b) = b - log(2u + 1) - log(1 + u) with u = e^b, so
    # dL/db = 1 - 2u/(2u + 1) - u/(1 + u) = 0  <=>  1 + u = u (2u + 1)  <=>  u^2 = 1/2,
    # b = -log(2) / 2, and -L'' = 2u/(2u + 1)^2 + u/(1 + u)^2 = 2 sqrt2 / (3 + 2 sqrt2).
    Xd = np.array([[1.0, 0.0, 1.0]])
    y = np.array([1.0, 2.0, 3.0])
    ev = np.array([1, 1, 0], np.int32)
    b, cov, it, conv = oracle.newton(oracle.Matrix.dense(Xd), y, ev, [0], gtol=1e-14)
    assert conv
    assert b[0] == pytest.approx(-0.5 * np.log(2.0), rel=1e-13)
    r2 = np.sqrt(2.0)
    assert cov[0, 0] == pytest.approx((3.0 + 2.0 * r2) / (2.0 * r2), rel=1e-12)


def test_lambda_max_with_unpenalised_columns():
    d, Xd, X = _problem(n=260, p=12, q=3, seed=64)
    rng = np.random.default_rng(5)
    pf = _weights(12, 3, rng)
    lm, bu = oracle.lambda_max_pf(X, d.time, d.event, pf)
    free = np.flatnonzero(pf == 0)
    # brute force: the sub-problem by BFGS on the O(n^2) likelihood, then max |g_j| / pf_j
    def nll(z):
        b = np.zeros(X.p)
        b[free] = z
        return -brute.loglik(Xd.T @ b, d.time, d.event), -brute.gradient(Xd, b, d.time, d.event)[free]
    res = scipy.optimize.minimize(nll, np.zeros(free.size), jac=True, method="BFGS", options=dict(gtol=1e-12))
    np.testing.assert_allclose(bu, res.x, rtol=1e-6, atol=1e-9)
    b = np.zeros(X.p)
    b[free] = res.x
    g = brute.gradient(Xd, b, d.time, d.event)
    pen = pf > 0
    assert lm == pytest.approx(np.max(np.abs(g[pen]) / pf[pen]), rel=1e-7)
    # no unpenalised column: the closed form at beta = 0, weighted
    pf1 = np.where(pf > 0, pf, 1.0)
    lm1, _ = oracle.lambda_max_pf(X, d.time, d.event, pf1)
    g0 = brute.gradient(Xd, np.zeros(X.p), d.time, d.event)
    assert lm1 == pytest.approx(np.max(np.abs(g0) / pf1), rel=1e-12)
    # just above lambda_max the penalised coefficients stay zero; just below, the arg max enters
    sigma = 1.0 / (2.0 * oracle.opnorm2(X)[0])
    hi, _, _, _ = oracle.fit(X, d.time, d.event, lm * (1 + 1e-6), sigma, max_iter=40000, tol=1e-15, pf=pf)
    assert np.all(hi[pen] == 0.0)
    np.testing.assert_allclose(hi[free], bu, rtol=1e-5)
    lo, _, _, _ = oracle.fit(X, d.time, d.event, lm * (1 - 1e-2), sigma, max_iter=40000, tol=1e-15, pf=pf)
    j = np.flatnonzero(pen)[np.argmax(np.abs(g[pen]) / pf[pen])]
    np.testing.assert_array_equal(np.flatnonzero(lo[pen] != 0), [np.flatnonzero(np.flatnonzero(pen) == j)[0]])


def test_penalty_factor_input_checks():
    d, Xd, X = _problem(n=60, p=5, q=1, seed=65)
    with pytest.raises(ValueError):
        oracle.fit(X, d.time, d.event, 1.0, 1e-3, max_iter=1, pf=np.full(X.p, -1.0))
    with pytest.raises(ValueError):
        oracle.lambda_max_pf(X, d.time, d.event, np.full(X.p, np.nan))
