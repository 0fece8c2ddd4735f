"""Pins of the oracle's Section 6 ranking (columns ordered by the largest
lambda at which they are nonzero, ties by |coefficient| on entry; a reading
breaks the remaining ties by column index): a worked case by hand, an
incremental construction on random paths, and invariances."""
import numpy as np
import pytest

import oracle


def test_rank_by_hand():
    path = np.zeros((3, 10), np.float32)
    path[0, 7] = -0.5    # the only column at the largest lambda
    path[1, 7] = -0.6
    path[1, 2] = 0.1     # enters at the second lambda, smaller |coef| than column 9
    path[1, 9] = -0.3
    path[2, 2] = 0.2
    path[2, 4] = 0.3     # enters at the third lambda
    path[2, 5] = -0.3    # same row and |coef| as column 4: column order
    entry, coef, order = oracle.rank_path(path)
    np.testing.assert_array_equal(order, [7, 9, 2, 4, 5])
    np.testing.assert_array_equal(entry, [-1, -1, 1, -1, 2, 2, -1, 0, -1, 1])
    np.testing.assert_array_equal(coef, np.float32([0, 0, 0.1, 0, 0.3, 0.3, 0, 0.5, 0, 0.3]))


def _incremental(path):
    """Walk the lambdas in order; the columns that are nonzero for the first
    time join in order of decreasing |coefficient|, then column index."""
    L, p = path.shape
    seen = set()
    out = []
    for l in range(L):
        new = [j for j in range(p) if path[l, j] != 0 and j not in seen]
        new.sort(key=lambda j: (-abs(float(path[l, j])), j))
        out += new
        seen.update(new)
    return out


@pytest.mark.parametrize("seed", range(20))
def test_rank_matches_incremental_construction(seed):
    rng = np.random.default_rng(seed)
    L, p = int(rng.integers(1, 7)), int(rng.integers(1, 40))
    path = np.zeros((L, p), np.float32)
    for l in range(L):
        on = rng.random(p) < 0.15 + 0.1 * l
        # few distinct magnitudes, so that ties on |coefficient| happen
        path[l, on] = rng.choice([-0.5, -0.25, 0.25, 0.5, 1.0], on.sum())
    entry, coef, order = oracle.rank_path(path)
    np.testing.assert_array_equal(order, _incremental(path))
    for j in range(p):
        rows = np.nonzero(path[:, j])[0]
        assert entry[j] == (rows[0] if rows.size else -1)
        assert coef[j] == (abs(path[rows[0], j]) if rows.size else 0)


def test_rank_invariances():
    rng = np.random.default_rng(5)
    path = (rng.standard_normal((5, 60)) * (rng.random((5, 60)) < 0.3)).astype(np.float32)
    _, _, o = oracle.rank_path(path)
    for q in (3.0 * path, -path, 0.5 * path):
        np.testing.assert_array_equal(oracle.rank_path(q)[2], o)
    # relabelling the columns relabels the ranking (no ties on |coefficient| here)
    perm = rng.permutation(60)
    _, _, op = oracle.rank_path(path[:, perm])
    np.testing.assert_array_equal(perm[op], o)


def test_rank_degenerate_paths():
    entry, coef, order = oracle.rank_path(np.zeros((4, 9), np.float32))
    assert order.size == 0 and np.all(entry == -1) and np.all(coef == 0)
    entry, coef, order = oracle.rank_path(np.float32([[0.0, -2.0, 1.0]]))
    np.testing.assert_array_equal(order, [1, 2])
    with pytest.raises(ValueError):
        oracle.rank_path(np.zeros((0, 3), np.float32))
