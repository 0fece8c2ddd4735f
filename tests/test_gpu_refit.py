"""GPU parity of the post-selection step of Section 6: ranking the columns a
lasso path selects, the unpenalised Newton refit on them with the covariates,
and the Wald statistics, through the C ABI, against the FP64 oracle's Newton
fit and inverse information (pinned in tests/test_oracle_penalty.py) and the
oracle's ranking (pinned in tests/test_oracle_rank.py).

The refit gathers the chosen genotype columns as FP32 values of (g - mu) s.
Against the oracle on those same FP32 values the coefficients, standard
errors and log likelihood agree to 1e-8 relative (both are exact Newton
solutions of the same problem, summed in different orders). Against the
oracle on the exact FP64 values they agree to 1e-5, the effect of rounding the
design to FP32.
"""
import math

import numpy as np
import pytest

import coxsim
import oracle
from tests.gpu_helpers import device_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402

Q = 11


@pytest.fixture(scope="module")
def prob():
    d, Z, gamma = coxsim.genotype_problem_with_covariates(3001, 400, 8, Q, 0.7, 5150, days=True)
    return d, Z


def _setup(prob, storage, with_cov=True):
    d, Z = prob
    ldx = (d.n + 15) // 16 * 16
    cox, M = device_problem(d, storage, ldx=ldx)
    if with_cov:
        Zd = torch.from_numpy(Z).cuda()
        cox.set_covariates(Zd)
        cox._keep = Zd
    return cox, M


def _oracle_refit(d, Z, Xrows, with_cov=True):
    """Newton on the dense FP64 matrix whose rows are the given design columns (+ Z)."""
    rows = [Xrows] + ([Z.astype(np.float64)] if with_cov else [])
    Mo = oracle.Matrix.dense(np.vstack(rows))
    b, cov, it, conv = oracle.newton(Mo, d.time, d.event, np.arange(Mo.p), gtol=1e-11, maxit=100)
    assert conv
    L, _ = oracle.loglik(oracle.xbeta(Mo, b), d.time, d.event)
    return b, np.sqrt(np.diag(cov)), L


@pytest.mark.parametrize("storage", ["f32", "int8", "fp8"])
def test_refit_matches_oracle_newton(prob, storage):
    d, Z = prob
    cox, M = _setup(prob, storage)
    cols = np.array(sorted(set(d.causal.tolist()) | {3, 77, 250}), np.int64)
    coef, se, pv, L, it, st = cox.refit(cols, gtol=1e-9)
    assert st == P.OK and it >= 2
    # the same FP32 design values the GPU gathers
    X32 = M.to_dense64()[cols].astype(np.float32).astype(np.float64)
    bo, seo, Lo = _oracle_refit(d, Z, X32)
    np.testing.assert_allclose(coef, bo, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(se, seo, rtol=1e-8)
    assert L == pytest.approx(Lo, rel=1e-12)
    z = bo / seo
    want_p = np.array([math.erfc(abs(v) / math.sqrt(2.0)) for v in z])
    np.testing.assert_allclose(pv, want_p, rtol=1e-6, atol=1e-300)
    # against the exact FP64 design: the FP32 rounding of x~ only
    be, see, _ = _oracle_refit(d, Z, M.to_dense64()[cols])
    np.testing.assert_allclose(coef, be, rtol=1e-5, atol=1e-7)
    np.testing.assert_allclose(se, see, rtol=1e-5)


def test_refit_covariates_only_and_without_covariates(prob):
    d, Z = prob
    cox, M = _setup(prob, "f32")
    coef, se, pv, L, it, st = cox.refit([])
    bo, seo, Lo = _oracle_refit(d, Z, np.zeros((0, d.n)))
    assert st == P.OK
    np.testing.assert_allclose(coef, bo, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(se, seo, rtol=1e-8)
    cox0, _ = _setup(prob, "f32", with_cov=False)
    cols = d.causal[:3]
    coef0, se0, _, L0, _, st0 = cox0.refit(cols)
    bo0, seo0, Lo0 = _oracle_refit(d, Z, M.to_dense64()[cols], with_cov=False)
    assert st0 == P.OK and coef0.shape == (3,)
    np.testing.assert_allclose(coef0, bo0, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(se0, seo0, rtol=1e-8)
    assert L0 == pytest.approx(Lo0, rel=1e-12)


def test_refit_spans_several_factor_blocks(prob):
    """211 coefficients: six full 32-column blocks of the blocked Cholesky and
    the triangular solves, and a ragged tail of 19; Newton to convergence."""
    d, Z = prob
    cox, M = _setup(prob, "fp8")
    cols = np.sort(np.random.default_rng(31).choice(d.p, 200, replace=False))
    coef, se, pv, L, it, st = cox.refit(cols, gtol=1e-9)
    assert st == P.OK and coef.shape == (211,)
    X32 = M.to_dense64()[cols].astype(np.float32).astype(np.float64)
    bo, seo, Lo = _oracle_refit(d, Z, X32)
    assert np.abs(coef - bo).max() <= 1e-7 * np.abs(bo).max()
    np.testing.assert_allclose(se, seo, rtol=1e-7)
    assert L == pytest.approx(Lo, rel=1e-12)


def test_refit_at_the_column_limit():
    """COX_MAX_REFIT = 1024 coefficients (1013 SNPs + 11 covariates, 32 full
    blocks): one Newton step from zero, then the standard errors at the new
    point, against the oracle taking the same step."""
    d, Z, _ = coxsim.genotype_problem_with_covariates(4000, 1100, 8, Q, 0.7, 777, days=True)
    cox, M = device_problem(d, "int8", ldx=4000)
    Zd = torch.from_numpy(Z).cuda()
    cox.set_covariates(Zd)
    cox._keep = Zd
    cols = np.arange(P.MAX_REFIT - Q)
    coef, se, pv, L, it, st = cox.refit(cols, max_iter=1, gtol=1e-11)
    assert st == P.ERR_NOT_CONVERGED and it == 1
    X32 = M.to_dense64()[cols].astype(np.float32).astype(np.float64)
    Mo = oracle.Matrix.dense(np.vstack([X32, Z.astype(np.float64)]))
    bo, cov, ito, conv = oracle.newton(Mo, d.time, d.event, np.arange(Mo.p), maxit=1, gtol=1e-11)
    assert ito == 1 and not conv
    assert np.abs(coef - bo).max() <= 1e-7 * np.abs(bo).max()
    np.testing.assert_allclose(se, np.sqrt(np.diag(cov)), rtol=1e-7)
    Lo, _ = oracle.loglik(oracle.xbeta(Mo, bo), d.time, d.event)
    assert L == pytest.approx(Lo, rel=1e-12)


def _dense_cox(X, time, event):
    Xd = torch.from_numpy(X).cuda()
    cox = P.Cox(Xd, time, event, n=X.shape[1])
    cox._keep = Xd
    return cox


def test_refit_one_tie_group():
    """Every subject at the same time: one tie group, so the second Hessian
    term has a single row (the whole cohort's risk-set sums)."""
    rng = np.random.default_rng(8)
    n, p = 2000, 6
    X = rng.standard_normal((p, n)).astype(np.float32)
    time = np.full(n, 5.0)
    event = (rng.random(n) < 0.4).astype(np.int32)
    cox = _dense_cox(X, time, event)
    coef, se, pv, L, it, st = cox.refit(np.arange(p), gtol=1e-10)
    assert st == P.OK
    Mo = oracle.Matrix.dense(X.astype(np.float64))
    bo, cov, _, conv = oracle.newton(Mo, time, event, np.arange(p), gtol=1e-11, maxit=100)
    assert conv
    np.testing.assert_allclose(coef, bo, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(se, np.sqrt(np.diag(cov)), rtol=1e-8)
    # the closed form of the tied score at the solution: sum over events of x_i
    # minus d times the exp-weighted mean of x over everyone
    eta = X.astype(np.float64).T @ coef
    wgt = np.exp(eta - eta.max())
    score = X[:, event == 1].astype(np.float64).sum(axis=1) - event.sum() * (X.astype(np.float64) @ wgt) / wgt.sum()
    assert np.abs(score).max() <= 1e-8


def test_refit_without_events_is_not_positive_definite():
    """No events: no event groups (an empty second term) and a zero first
    term, so the information matrix is 0 and the factorisation reports it."""
    rng = np.random.default_rng(9)
    n, p = 700, 4
    X = rng.standard_normal((p, n)).astype(np.float32)
    cox = _dense_cox(X, rng.random(n), np.zeros(n, np.int32))
    with pytest.raises(P.CoxError) as ei:
        cox.refit(np.arange(p))
    assert ei.value.status == P.ERR_NUMERIC


def test_refit_from_a_start_and_iteration_cap(prob):
    d, Z = prob
    cox, M = _setup(prob, "int8")
    cols = d.causal[:4]
    full, *_ = cox.refit(cols, gtol=1e-9)
    # from the solution itself: no step needed
    again, se, pv, L, it, st = cox.refit(cols, coef0=full, gtol=1e-6)
    assert st == P.OK and it == 0
    np.testing.assert_array_equal(again, full)
    # one step from zero is not enough at this tolerance
    one = cox.refit(cols, max_iter=1, gtol=1e-12)
    assert one[5] == P.ERR_NOT_CONVERGED and one[4] == 1


def test_refit_argument_checks(prob):
    d, Z = prob
    cox, M = _setup(prob, "f32", with_cov=False)
    for bad in ([1, 1], [-1], [d.p], []):
        with pytest.raises(P.CoxError) as ei:
            cox.refit(bad)
        assert ei.value.status == P.ERR_INVALID_ARG
    with pytest.raises(P.CoxError) as ei:
        cox.refit([0], coef0=[np.nan])
    assert ei.value.status == P.ERR_INVALID_ARG


def test_rank_path_by_hand(prob):
    d, Z = prob
    cox, M = _setup(prob, "f32", with_cov=False)
    path = np.zeros((3, d.p), np.float32)
    path[0, 7] = -0.5    # enters first
    path[1, 7] = -0.6
    path[1, 2] = 0.1     # second row, smaller |coef| than column 9
    path[1, 9] = -0.3
    path[2, 2] = 0.2
    path[2, 4] = 0.3     # third row
    path[2, 5] = 0.3     # tie with column 4 on |coef|: index order
    entry, coef, order = cox.rank_path(torch.from_numpy(path).cuda())
    np.testing.assert_array_equal(order, [7, 9, 2, 4, 5])
    e_o, c_o, o_o = oracle.rank_path(path)
    np.testing.assert_array_equal(order, o_o)
    np.testing.assert_array_equal(entry, e_o)
    np.testing.assert_array_equal(coef, c_o)
    assert entry[7] == 0 and entry[2] == 1 and entry[4] == 2 and entry[0] == -1
    assert coef[9] == np.float32(0.3) and coef[7] == np.float32(0.5)


def test_section6_protocol_end_to_end(prob):
    """Unpenalised covariates, a decreasing lambda sequence to the lag-10 rule,
    the ranking, the refit on the entered SNPs and a Bonferroni cut."""
    d, Z = prob
    cox, M = _setup(prob, "fp8")
    lm = cox.lambda_max()
    lams = lm * np.geomspace(0.95, 0.35, 8)
    path, iters, obj, st = cox.fit_sequence(lams, max_iter=3000, tol=1e-5, lag=10)
    assert st == P.OK
    entry, coef, order = cox.rank_path(path)
    ref_entry, ref_coef, ref_order = oracle.rank_path(path.cpu().numpy()[:, : d.p])
    np.testing.assert_array_equal(entry, ref_entry)
    np.testing.assert_array_equal(coef, ref_coef)
    np.testing.assert_array_equal(order, ref_order)
    assert 0 < order.size <= 60
    b, se, pv, L, it, st = cox.refit(order, gtol=1e-9)
    assert st == P.OK
    X32 = M.to_dense64()[order].astype(np.float32).astype(np.float64)
    bo, seo, _ = _oracle_refit(d, Z, X32)
    np.testing.assert_allclose(b, bo, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(se, seo, rtol=1e-8)
    keep = order[pv[: order.size] < 0.01 / order.size]
    strong = d.causal[np.abs(d.beta_true[d.causal]) > 0.4]
    print(f"{order.size} SNPs entered; {keep.size} pass Bonferroni; strong causal {list(strong)} -> kept "
          f"{sorted(set(strong) & set(keep))}")
    assert set(strong) <= set(keep)


def test_refit_is_deterministic(prob):
    """Every sum of the refit runs in a fixed order: two calls agree bit for bit."""
    d, Z = prob
    cox, M = _setup(prob, "fp8")
    cols = np.sort(np.random.default_rng(5).choice(d.p, 90, replace=False))
    first = cox.refit(cols, gtol=1e-9)
    second = cox.refit(cols, gtol=1e-9)
    for a, b in zip(first[:3], second[:3]):
        np.testing.assert_array_equal(a, b)
    assert first[3] == second[3] and first[4] == second[4]
