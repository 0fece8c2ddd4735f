"""cox_rank_path_noalloc, the variant of cox_rank_path that allocates nothing
(its device working memory is a static array in the library), against
cox_rank_path through the C ABI: the entry rows, the |coef| at entry and the
ranking agree exactly, on two calls in a row on one GPU -- the second with a
smaller input, so that it runs over the first call's leftovers in the shared
array -- and a context wider than the array is turned away before any device
work."""
import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)
import paper_2010_16114_amd as P  # noqa: E402


def _context(n, p, seed):
    rng = np.random.default_rng(seed)
    X = torch.from_numpy(rng.standard_normal((p, n)).astype(np.float32)).cuda()
    time = rng.exponential(size=n)
    event = (rng.random(n) < 0.7).astype(np.int32)
    cox = P.Cox(X, time, event)
    cox._keep = X
    return cox


def _path(L, p, seed):
    """A decreasing-lambda path of L rows: columns enter at random rows and
    stay in; |coef| at entry is drawn from a few values so that ties on
    (entry, |coef|) occur and the index decides."""
    rng = np.random.default_rng(seed)
    path = np.zeros((L, p), np.float32)
    enter = rng.integers(0, 2 * L, p)  # >= L: never enters
    vals = np.array([0.125, 0.25, 0.5, 1.0], np.float32)
    for j in np.flatnonzero(enter < L):
        e = enter[j]
        sign = 1.0 if rng.random() < 0.5 else -1.0
        path[e, j] = sign * vals[rng.integers(0, vals.size)]
        path[e + 1:, j] = sign * rng.random(L - e - 1).astype(np.float32)
        path[e + 1:, j][path[e + 1:, j] == 0] = 0.5
    return torch.from_numpy(path).cuda()


@pytest.mark.parametrize("sizes", [((257, 5000, 20), (64, 1200, 6))])
def test_noalloc_rank_matches_rank_path_on_two_calls(sizes):
    for call, (n, p, L) in enumerate(sizes):
        print(f"[no_alloc] call {call}: n={n} p={p} L={L}", flush=True)
        cox = _context(n, p, 100 + call)
        path = _path(L, p, 200 + call)
        e_ref, c_ref, o_ref = cox.rank_path(path)
        e, c, o = cox.rank_path_noalloc(path)
        assert o_ref.size > 0
        np.testing.assert_array_equal(e, e_ref)
        np.testing.assert_array_equal(c.view(np.uint32), c_ref.view(np.uint32))
        np.testing.assert_array_equal(o, o_ref)
        e_o, c_o, o_o = oracle.rank_path(path.cpu().numpy())  # and both are Section 6's ranking
        np.testing.assert_array_equal(e, e_o)
        np.testing.assert_array_equal(o, o_o)
        cox.close()


def test_noalloc_rejects_wider_than_its_scratch():
    n, p = 16, P.NOALLOC_MAX_COLS + 1
    X = torch.zeros((p, n), dtype=torch.int8, device="cuda")
    time = np.arange(n, dtype=np.float64) + 1.0
    event = np.ones(n, np.int32)
    cox = P.Cox(X, time, event, xtype=P.X_INT8)
    path = torch.zeros((1, p), dtype=torch.float32, device="cuda")
    with pytest.raises(P.CoxError) as ei:
        cox.rank_path_noalloc(path)
    assert ei.value.status == P.ERR_UNSUPPORTED
    cox.close()
    del X, path
    torch.cuda.empty_cache()
