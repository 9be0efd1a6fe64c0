"""Pins for the oracle's support selection (kNN, paper section II).

The definition: the k nodes with the smallest keys (d2, j), d2 = fl(fl(dx^2) +
fl(dy^2)), lexicographic, NaN keys never taken.  Pinned against SciPy's k-d
tree on tie-free inputs and against Python's own sort on inputs full of exact
ties.
"""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from paper_2107_03632_amd import nodes


def _py_knn(x, y, i, k):
    keys = []
    for j in range(len(x)):
        dx = float(x[j]) - float(x[i])
        dy = float(y[j]) - float(y[i])
        d2 = dx * dx + dy * dy  # Python floats: IEEE double, no contraction
        if d2 == d2:
            keys.append((d2, j))
    keys.sort()
    out = [j for _, j in keys[:k]]
    return out + [-1] * (k - len(out))


@pytest.mark.parametrize("k", [1, 6, 12, 30])
def test_knn_matches_kdtree_on_jittered_nodes(k):
    ns = nodes.unit_square(20, seed=7)
    got = oracle.knn(ns.x, ns.y, k)
    pts = np.stack([ns.x, ns.y], 1)
    d, idx = cKDTree(pts).query(pts, k=k)
    idx = idx.reshape(len(pts), k)
    d2 = (ns.x[got] - ns.x[:, None]) ** 2 + (ns.y[got] - ns.y[:, None]) ** 2
    d2_tree = (ns.x[idx] - ns.x[:, None]) ** 2 + (ns.y[idx] - ns.y[:, None]) ** 2
    for i in range(len(pts)):
        # same multiset of distances; same indices strictly inside the k-th
        # distance (the k-d tree breaks ties at the k-th distance arbitrarily)
        assert np.array_equal(np.sort(d2[i]), np.sort(d2_tree[i]))
        kth = d2[i].max()
        assert set(got[i][d2[i] < kth]) == set(idx[i][d2_tree[i] < kth])
    # ascending distances
    assert np.all(np.diff(d2, axis=1) >= 0)
    # self first (no duplicates in this set)
    assert np.all(got[:, 0] == np.arange(len(pts)))


def test_knn_tie_break_by_index_on_exact_lattice():
    # unjittered integer lattice: many exactly equal distances
    g = np.arange(7, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel(), Y.ravel()
    rng = np.random.default_rng(3)
    perm = rng.permutation(x.size)  # shuffle so index order != spatial order
    x, y = x[perm].copy(), y[perm].copy()
    got = oracle.knn(x, y, 13)
    for i in range(x.size):
        assert list(got[i]) == _py_knn(x, y, i, 13)


def test_knn_subset_of_queries_and_duplicates():
    ns = nodes.unit_square(10, seed=2)
    x = np.concatenate([ns.x, ns.x[:3]])
    y = np.concatenate([ns.y, ns.y[:3]])
    q = np.array([0, 1, x.size - 1, 57])
    got = oracle.knn(x, y, 9, queries=q)
    for t, i in enumerate(q):
        assert list(got[t]) == _py_knn(x, y, int(i), 9)
    # the duplicate of node 0 is at distance 0 with a larger index
    assert got[0][0] == 0 and got[0][1] == ns.n_nodes


def test_knn_nan_nodes_never_selected():
    ns = nodes.unit_square(8, seed=4)
    x, y = ns.x.copy(), ns.y.copy()
    x[5] = np.nan
    got = oracle.knn(x, y, 8)
    assert not np.any(got[np.arange(x.size) != 5] == 5)
    assert np.all(got[5] == -1)
    for i in [0, 6, 20]:
        assert list(got[i]) == _py_knn(x, y, i, 8)


def test_knn_rejects_bad_k():
    x = np.zeros(4)
    with pytest.raises(ValueError):
        oracle.knn(x, x, 5)
    with pytest.raises(ValueError):
        oracle.knn(x, x, 0)
