"""Pin for the oracle's adjoint (reverse mode of the weights map): central
finite differences of L = sum g_ij w_ij with the supports held fixed,
evaluated only over the stencils a perturbed node touches.

m = 2, 4: two-point central differences with step 1e-6 h.  m = 6: the
round-off floor of a difference quotient is about eps * cond(M) * h / step,
and order-6 boundary stencils reach cond ~1e7, so the step is 1e-4 h with the
four-point central stencil (truncation error O(step^4)) instead.
"""

import numpy as np
import pytest

import oracle
from paper_2107_03632_amd import nodes

NFM = {2: 12, 4: 30, 6: 56}


def _local_loss(x, y, nbr, G, m, n, rows):
    w, st = oracle.weights(x, y, nbr, m=m, n=n, rows=rows)
    assert np.all(st == 0)
    return float(np.sum(G[rows] * w))


@pytest.mark.parametrize("m", [2, 4, 6])
def test_adjoint_matches_central_differences(m):
    ns = nodes.annulus(1500, seed=8)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    G = nodes.gaussian_cotangent(ns.n_nodes, n, seed=55)
    gx, gy, failed = oracle.adjoint(ns.x, ns.y, nbr, G, m=m, n=n)
    assert failed == 0
    d = (1e-4 if m == 6 else 1e-6) * ns.h
    taps = ((2, -1 / 12), (1, 8 / 12), (-1, -8 / 12), (-2, 1 / 12)) if m == 6 \
        else ((1, 0.5), (-1, -0.5))
    rng = np.random.default_rng(1)
    sample = rng.choice(ns.n_nodes, size=12, replace=False)
    adj, fd = [], []
    for p in sample:
        rows = np.unique(np.concatenate([[p], np.nonzero(np.any(nbr == p, axis=1))[0]]))
        for coord, g in ((0, gx), (1, gy)):
            acc = 0.0
            for sgn, c in taps:
                x, y = ns.x.copy(), ns.y.copy()
                (x if coord == 0 else y)[p] += sgn * d
                acc += c * _local_loss(x, y, nbr, G, m, n, rows)
            fd.append(acc / d)
            adj.append(g[p])
    adj, fd = np.array(adj), np.array(fd)
    err = np.abs(adj - fd).max() / np.abs(fd).max()
    assert err <= 1e-6, err


def test_adjoint_self_node_and_translation_invariance():
    # L depends on coordinate differences only, so the gradient sums to zero
    ns = nodes.unit_square(10, seed=12)
    nbr = oracle.knn(ns.x, ns.y, 12)
    G = nodes.gaussian_cotangent(ns.n_nodes, 12, seed=3)
    gx, gy, failed = oracle.adjoint(ns.x, ns.y, nbr, G, m=2, n=12)
    assert failed == 0
    assert abs(gx.sum()) <= 1e-9 * np.abs(gx).sum()
    assert abs(gy.sum()) <= 1e-9 * np.abs(gy).sum()


def test_adjoint_restricted_to_the_stencils_of_sampled_nodes():
    # the gradient at a node only gathers the stencils that name it, so the
    # adjoint over those stencils alone gives the same bits there
    ns = nodes.unit_square(14, seed=12)
    nbr = oracle.knn(ns.x, ns.y, 30)
    G = nodes.gaussian_cotangent(ns.n_nodes, 30, seed=3)
    gx, gy, failed = oracle.adjoint(ns.x, ns.y, nbr, G, m=4, n=30)
    assert failed == 0
    sample = np.array([3, 50, 111, 170])
    rows = np.unique(np.concatenate([sample, np.nonzero(np.isin(nbr, sample).any(axis=1))[0]]))
    assert rows.size < ns.n_nodes
    gxr, gyr, failed = oracle.adjoint(ns.x, ns.y, nbr, G, m=4, n=30, rows=rows)
    assert failed == 0
    assert np.array_equal(gxr[sample], gx[sample]) and np.array_equal(gyr[sample], gy[sample])
    others = np.setdiff1d(np.arange(ns.n_nodes), rows)
    assert np.any(gxr[others] != gx[others])
