"""GPU parity of nonnegative matrix factorisation (Section 5.1) through the C
ABI (include/nmf.h) against the FP64 NMF oracle (pinned in
tests/test_oracle_nmf.py), from the same start, iterate by iterate.

Both sides keep the factors in FP64 and form every product with the FP32 X in
FP64, so they differ only in the order of the sums: after K iterations the
factors agree to 1e-9 of their largest entry and the objective to 1e-10
relative (the multiplicative update amplifies rounding differences only
mildly over tens of iterations).
"""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402

FAC_TOL = 1e-9
OBJ_TOL = 1e-10


def _data(m, n, r, seed, pad=0):
    rng = np.random.default_rng(seed)
    X = rng.random((m, n)).astype(np.float32)
    Vt = rng.random((r, m))
    W = rng.random((r, n))
    Xd = torch.zeros((m, n + pad), dtype=torch.float32)
    Xd[:, :n] = torch.from_numpy(X)
    return X, Vt, W, Xd.cuda()


def _rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


# (n, row padding): 777 + 5 leaves rows of X unaligned, so the passes stage
# through LDS; 778 + 2 gives 16-byte-aligned rows and even factor lengths,
# so they load straight from memory, with a ragged last step in both
# directions (m = 1000 rows, 778 columns)
LAYOUTS = {"lds": (777, 5), "direct": (778, 2)}


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
@pytest.mark.parametrize("r", [5, 20, 40, 60])
@pytest.mark.parametrize("algo", [P.NMF_MULTIPLICATIVE, P.NMF_APG])
def test_nmf_matches_oracle(r, algo, layout):
    m, K = 1000, 20
    n, pad = LAYOUTS[layout]
    X, Vt0, W0, Xd = _data(m, n, r, 10 + r, pad=pad)
    nmf = P.NMF(Xd, r, n=n)
    Vt = torch.from_numpy(Vt0).cuda()
    W = torch.from_numpy(W0).cuda()
    f = nmf.run(Vt, W, algo, K)
    Vo, Wo, tr = oracle.nmf_run(X, Vt0, W0, algo, K)
    assert _rel(Vt.cpu().numpy(), Vo) <= FAC_TOL
    assert _rel(W.cpu().numpy(), Wo) <= FAC_TOL
    assert f == pytest.approx(tr[-1], rel=OBJ_TOL)
    assert tr[-1] < tr[0]


def test_objective_without_iterations_and_continuation():
    m, n, r = 513, 300, 7
    X, Vt0, W0, Xd = _data(m, n, r, 3)
    nmf = P.NMF(Xd, r)
    Vt = torch.from_numpy(Vt0).cuda()
    W = torch.from_numpy(W0).cuda()
    assert nmf.run(Vt, W, P.NMF_APG, 0) == pytest.approx(oracle.nmf_objective(X, Vt0, W0), rel=1e-12)
    # 3 + 4 iterations in two calls equal 7 in one
    nmf.run(Vt, W, P.NMF_MULTIPLICATIVE, 3, want_obj=False)
    f = nmf.run(Vt, W, P.NMF_MULTIPLICATIVE, 4)
    Vo, Wo, tr = oracle.nmf_run(X, Vt0, W0, P.NMF_MULTIPLICATIVE, 7)
    assert _rel(Vt.cpu().numpy(), Vo) <= FAC_TOL and _rel(W.cpu().numpy(), Wo) <= FAC_TOL
    assert f == pytest.approx(tr[-1], rel=OBJ_TOL)


@pytest.mark.parametrize("r", [20, 60])
def test_full_size_10000_square(r):
    """The paper's GPU shape, 10,000 x 10,000 at r = 20 and 60 (the largest of
    its ranks): two iterations of each algorithm against the oracle, every
    entry of both factors."""
    m = n = 10000
    X, Vt0, W0, Xd = _data(m, n, r, 77)
    nmf = P.NMF(Xd, r)
    for algo in (P.NMF_MULTIPLICATIVE, P.NMF_APG):
        Vt = torch.from_numpy(Vt0).cuda()
        W = torch.from_numpy(W0).cuda()
        f = nmf.run(Vt, W, algo, 2)
        Vo, Wo, tr = oracle.nmf_run(X, Vt0, W0, algo, 2)
        assert _rel(Vt.cpu().numpy(), Vo) <= FAC_TOL
        assert _rel(W.cpu().numpy(), Wo) <= FAC_TOL
        assert f == pytest.approx(tr[-1], rel=OBJ_TOL)


def test_nmf_argument_checks():
    X, Vt0, W0, Xd = _data(64, 40, 3, 5)
    with pytest.raises(P.CoxError) as ei:
        P.NMF(Xd, P.NMF_MAX_RANK + 1)
    assert ei.value.status == P.ERR_INVALID_ARG
    nmf = P.NMF(Xd, 3)
    Vt = torch.from_numpy(Vt0).cuda()
    W = torch.from_numpy(W0).cuda()
    with pytest.raises(P.CoxError) as ei:
        nmf.run(Vt, W, 2, 1)
    assert ei.value.status == P.ERR_INVALID_ARG
    with pytest.raises(P.CoxError) as ei:
        nmf.run(Vt, W, P.NMF_APG, 1, eps=-1.0)
    assert ei.value.status == P.ERR_INVALID_ARG


@pytest.mark.parametrize("layout", sorted(LAYOUTS))
def test_nmf_is_deterministic(layout):
    """The split partials are added in a fixed order: two runs from the same
    start agree bit for bit."""
    m, r = 1000, 20
    n, pad = LAYOUTS[layout]
    X, Vt0, W0, Xd = _data(m, n, r, 404, pad=pad)
    nmf = P.NMF(Xd, r, n=n)
    out = []
    for _ in range(2):
        Vt = torch.from_numpy(Vt0).cuda()
        W = torch.from_numpy(W0).cuda()
        f = nmf.run(Vt, W, P.NMF_APG, 10)
        out.append((Vt.cpu().numpy(), W.cpu().numpy(), f))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]
