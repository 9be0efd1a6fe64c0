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


@pytest.mark.parametrize("m,n", [(2, 12), (4, 30), (6, 56), (2, 20), (4, 40), (6, 60)])
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


@pytest.mark.parametrize("m,n", [(2, 12), (4, 30)])
def test_derivative_of_phs_interpolant(m, n):
    """w . f equals d/dx (d/dy) of s_f at the centre, where s_f is the r^3 +
    monomial interpolant of f on the stencil, taken by 30-digit numerical
    differentiation.  Polynomial reproduction holds whatever the r^3 part of
    the right-hand side is; this pins that part (its constant, sign and
    which offset component it takes)."""
    import mpmath
    ns = nodes.unit_square(12, seed=17)
    nbr = oracle.knn(ns.x, ns.y, n)
    rng = np.random.default_rng(6)
    ex = monos(m)
    for i in [30, 77]:
        idx = nbr[i]
        px, py = ns.x[idx], ns.y[idx]
        cx, cy = ns.x[i], ns.y[i]
        f = rng.standard_normal(n)
        A = np.sqrt((px[:, None] - px[None]) ** 2 + (py[:, None] - py[None]) ** 2) ** 3
        P = np.array([[(a_ - cx) ** e[0] * (b_ - cy) ** e[1] for e in ex]
                      for a_, b_ in zip(px, py)])
        M = np.block([[A, P], [P.T, np.zeros((len(ex), len(ex)))]])
        coef = np.linalg.solve(M, np.concatenate([f, np.zeros(len(ex))]))
        with mpmath.workdps(30):
            def s_f(X, Y):
                acc = mpmath.mpf(0)
                for k in range(n):
                    acc += coef[k] * mpmath.sqrt((X - px[k]) ** 2 + (Y - py[k]) ** 2) ** 3
                for j, e in enumerate(ex):
                    acc += coef[n + j] * (X - cx) ** e[0] * (Y - cy) ** e[1]
                return acc
            X0, Y0 = mpmath.mpf(cx), mpmath.mpf(cy)
            ddx = mpmath.diff(lambda t: s_f(t, Y0), X0, 1)
            ddy = mpmath.diff(lambda t: s_f(X0, t), Y0, 1)
        for op, want in ((oracle.D_DX, float(ddx)), (oracle.D_DY, float(ddy))):
            w, st = oracle.weights_op(ns.x, ns.y, nbr, m, n, op, rows=[i])
            assert st[0] == 0
            got = float(np.dot(w[0, :n], f))
            assert abs(got - want) <= 1e-8 * np.abs(w[0, :n] * f).sum(), (op, got, want)
