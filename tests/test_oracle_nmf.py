"""Pins of the NMF oracle (Section 5.1) against what the mathematics fixes.

A plausible slip (sigma without its factor 2 or the square of the norm, the W
update taking the old V, a swapped product, a dropped eps) fails at least one:
  * a 1 x 1 problem whose two updates are worked out by hand;
  * monotone decrease of f for both updates (Lee and Seung's theorem for the
    multiplicative one; the APG step is at most 1 / Lipschitz);
  * an exact nonnegative factorisation is a fixed point of the multiplicative
    update (up to eps);
  * the objective against its expansion ||X||^2 - 2<V'X, W> + <V'V, W W'>;
  * the KKT conditions of the nonnegatively constrained problem after a long
    APG run: V, W >= 0, gradient >= 0, complementary slackness;
  * recovery of an exactly rank-2 nonnegative X (f -> 0).
"""
import numpy as np
import pytest

import oracle

MU, APG = oracle.NMF_MU, oracle.NMF_APG


def test_one_by_one_by_hand():
    # x = 2, v = 1, w = 1, eps = 0.
    X = np.array([[2.0]], np.float32)
    V, W = np.array([[1.0]]), np.array([[1.0]])
    # multiplicative: v' = v (x w) / (v w^2) = 2; w' = w (v' x) / (v'^2 w) = 4 / 4 = 1
    v, w, tr = oracle.nmf_run(X, V, W, MU, 1, eps=0.0)
    assert v[0, 0] == 2.0 and w[0, 0] == 1.0
    assert tr[0] == 1.0 and tr[1] == 0.0
    # APG: sigma = 1 / (2 w^4) = 1/2, v' = 1 - (1/2)(1 - 2) = 3/2;
    # tau = 1 / (2 v'^4) = 8/81, w' = 1 - (8/81)(v'^2 w - v' x) = 1 + (8/81)(3/4) = 29/27
    v, w, tr = oracle.nmf_run(X, V, W, APG, 1, eps=0.0)
    assert v[0, 0] == 1.5
    assert w[0, 0] == pytest.approx(29.0 / 27.0, rel=1e-15)
    assert tr[1] == pytest.approx((2.0 - 1.5 * 29.0 / 27.0) ** 2, rel=1e-14)
    # projection: a step that would go negative stops at 0 (x = 0, v = w = 1:
    # v' = 1 - (1/2)(1 - 0) = 1/2, tau = 1/(2 (1/2)^4) = 8, w' = max(0, 1 - 8 (1/4)) = 0)
    v, w, _ = oracle.nmf_run(np.array([[0.0]], np.float32), V, W, APG, 1, eps=0.0)
    assert v[0, 0] == 0.5 and w[0, 0] == 0.0


@pytest.mark.parametrize("algo", [MU, APG])
@pytest.mark.parametrize("seed", [0, 1])
def test_monotone_decrease(algo, seed):
    rng = np.random.default_rng(seed)
    m, n, r = 70, 53, 5
    X = rng.random((m, n)).astype(np.float32)
    _, _, tr = oracle.nmf_run(X, rng.random((r, m)), rng.random((r, n)), algo, 300)
    assert np.all(np.diff(tr) <= 1e-12 * tr[1:]), np.diff(tr).max()
    assert tr[-1] < 0.5 * tr[0]


def test_exact_factorisation_is_a_multiplicative_fixed_point():
    rng = np.random.default_rng(2)
    m, n, r = 40, 30, 3
    V = rng.integers(1, 4, size=(r, m)).astype(np.float64)   # V' with entries 1..3
    W = rng.integers(1, 4, size=(r, n)).astype(np.float64)
    X = (V.T @ W).astype(np.float32)                          # small integers: exact
    v, w, tr = oracle.nmf_run(X, V, W, MU, 3, eps=1e-10)
    assert np.abs(v - V).max() <= 1e-9 * V.max()
    assert np.abs(w - W).max() <= 1e-9 * W.max()
    assert tr[0] == 0.0


def test_objective_expansion():
    rng = np.random.default_rng(3)
    m, n, r = 33, 21, 4
    X = rng.random((m, n)).astype(np.float32)
    V, W = rng.random((r, m)), rng.random((r, n))
    Xd = X.astype(np.float64)
    want = (Xd ** 2).sum() - 2.0 * ((V @ Xd) * W).sum() + ((V @ V.T) * (W @ W.T)).sum()
    assert oracle.nmf_objective(X, V, W) == pytest.approx(want, rel=1e-12)


def test_apg_reaches_kkt():
    rng = np.random.default_rng(4)
    m, n, r = 25, 18, 3
    X = rng.random((m, n)).astype(np.float32)
    V, W, tr = oracle.nmf_run(X, rng.random((r, m)), rng.random((r, n)), APG, 60000, eps=1e-16)
    Xd = X.astype(np.float64)
    # gradients of f / 2 in V' and W
    GV = (W @ W.T) @ V - W @ Xd.T
    GW = (V @ V.T) @ W - V @ Xd
    assert V.min() >= 0 and W.min() >= 0
    scale = np.abs(W @ Xd.T).max()
    for F, G in ((V, GV), (W, GW)):
        assert G.min() >= -1e-6 * scale
        assert np.abs(F * G).max() <= 1e-6 * scale * F.max()


def test_recovers_exact_low_rank():
    rng = np.random.default_rng(5)
    m, n, r = 30, 24, 2
    X = (rng.random((r, m)).T @ rng.random((r, n))).astype(np.float32)
    # the APG step 1/(2 ||W W'||_F^2) is well below 1/Lipschitz, so APG creeps
    # along the flat directions: after 20,000 steps it sits near 2e-7 of ||X||^2
    for algo, rel in ((MU, 1e-7), (APG, 1e-6)):
        _, _, tr = oracle.nmf_run(X, rng.random((r, m)), rng.random((r, n)), algo, 20000, eps=1e-16)
        assert tr[-1] <= rel * (X.astype(np.float64) ** 2).sum(), (algo, tr[-1])
        assert tr[0] > 1e3 * tr[-1]
