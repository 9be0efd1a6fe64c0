"""Pins for the oracle's first-derivative weights (oracle.weights_op with
D_DX / D_DY): eq. (1) with the right-hand side [L phi_k; L p_j] of L = d/dx
or d/dy at the stencil's centre.

* polynomial reproduction: the weights differentiate every monomial of
  degree <= m exactly (up to rounding), which fixes the polynomial part of
  the right-hand side and the 1/s scaling;
* scale invariance: scaling every coordinate by a scales the weights by 1/a
  (a first derivative), not by 1/a^2;
* reflection: on an exact lattice with a support made of whole rings, the
  d/dx weights are odd under x -> -x and even under y -> -y;
* the Laplacian (op 0) is bit-identical to oracle.weights.
"""

import numpy as np
import pytest

import oracle
from paper_2107_03632_amd import nodes


def monos(m):
    return [(a, d - a) for d in range(m + 1) for a in range(d, -1, -1)]


@pytest.mark.parametrize("m,n", [(2, 12), (4, 30), (6, 56)])
@pytest.mark.parametrize("op", [oracle.D_DX, oracle.D_DY])
def test_derivative_reproduces_polynomials(m, n, op):
    ns = nodes.unit_square(20, seed=41)
    nbr = oracle.knn(ns.x, ns.y, n)
    rows = np.arange(0, ns.n_nodes, 23)
    full = np.zeros_like(nbr)
    full[rows] = nbr[rows]
    w, st = oracle.weights_op(ns.x, ns.y, full, m, n, op, rows=rows)
    assert np.all(st == 0)
    for t, i in enumerate(rows):
        dx = ns.x[nbr[i]] - ns.x[i]
        dy = ns.y[nbr[i]] - ns.y[i]
        for a, b in monos(m):
            vals = dx ** a * dy ** b
            got = float(np.dot(w[t], vals))
            want = 1.0 if (op == oracle.D_DX and (a, b) == (1, 0)) or \
                (op == oracle.D_DY and (a, b) == (0, 1)) else 0.0
            scale = float(np.abs(w[t] * vals).sum()) + 1.0
            assert abs(got - want) <= 1e-10 * scale, (i, a, b, got)


@pytest.mark.parametrize("op", [oracle.D_DX, oracle.D_DY])
def test_derivative_scale_invariance(op):
    ns = nodes.unit_square(16, seed=42)
    nbr = oracle.knn(ns.x, ns.y, 30)
    w1, _ = oracle.weights_op(ns.x, ns.y, nbr, 4, 30, op)
    a = 8.0  # a power of two: the scaled coordinates are exact
    w2, _ = oracle.weights_op(a * ns.x, a * ns.y, nbr, 4, 30, op)
    np.testing.assert_allclose(w2 * a, w1, rtol=1e-12, atol=1e-12 * np.abs(w1).max())


@pytest.mark.parametrize("m,n", [(2, 13), (4, 29)])
def test_derivative_reflection_symmetry(m, n):
    # 13 = 1 + 4 + 4 + 4 and 29 = 1 + 4 + 4 + 4 + 8 + 4 + 4: whole rings of an
    # exact lattice around an interior node, so the support is mirror symmetric
    ns = nodes.cell_centred_square(24, seed=0, jitter=0.0)
    nbr = oracle.knn(ns.x, ns.y, n)
    h = 1.0 / 24
    i = int(np.argmin((ns.x - 0.5 - h / 2) ** 2 + (ns.y - 0.5 - h / 2) ** 2))
    dx = np.round((ns.x[nbr[i]] - ns.x[i]) / h).astype(int)
    dy = np.round((ns.y[nbr[i]] - ns.y[i]) / h).astype(int)
    key = {(a, b): k for k, (a, b) in enumerate(zip(dx, dy))}
    assert all((-a, b) in key and (a, -b) in key for a, b in key)
    wx, _ = oracle.weights_op(ns.x, ns.y, nbr, m, n, oracle.D_DX)
    wy, _ = oracle.weights_op(ns.x, ns.y, nbr, m, n, oracle.D_DY)
    tol = 1e-10 * np.abs(wx[i]).max()
    for (a, b), k in key.items():
        assert abs(wx[i][k] + wx[i][key[(-a, b)]]) <= tol   # odd in x
        assert abs(wx[i][k] - wx[i][key[(a, -b)]]) <= tol   # even in y
        assert abs(wy[i][k] + wy[i][key[(a, -b)]]) <= tol   # odd in y
        assert abs(wy[i][k] - wy[i][key[(-a, b)]]) <= tol   # even in x


def test_laplacian_operator_is_the_weights():
    ns = nodes.unit_square(12, seed=43)
    nbr = oracle.knn(ns.x, ns.y, 30)
    w0, s0 = oracle.weights(ns.x, ns.y, nbr, m=4, n=30)
    w1, s1 = oracle.weights_op(ns.x, ns.y, nbr, 4, 30, oracle.LAPLACIAN)
    assert np.array_equal(w0, w1) and np.array_equal(s0, s1)
