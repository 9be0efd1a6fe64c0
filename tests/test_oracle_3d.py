"""Pins for the oracle's three-dimensional support selection and Laplacian
weights (oracle.knn3, oracle.weights3): eq. (1) with d = 3, phi = r^3 and
the monomials of degree <= m in x, y, z.

* kNN: SciPy's k-d tree on jittered nodes (distance multisets, and the index
  sets strictly inside the k-th distance); Python's own sort of the keys
  (d^2, j) on an exact cubic lattice full of ties, with a duplicate and a
  NaN node.
* weights: the Laplacian of the r^3 + monomial interpolant of random data
  by 30-digit numerical differentiation (pins lap r^3 = 12 r, the A block
  and the scaling); exact reproduction of every monomial of degree <= m
  (pins the monomial set and its right-hand side); scaling by a gives
  1/a^2; a rotation and translation of the node set leaves the weights
  unchanged; the status codes.
"""

import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle


def jittered_cube(q, seed, jitter=0.25):
    rng = np.random.default_rng(seed)
    g = (np.arange(q) + 0.5) / q
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    pts += rng.uniform(-jitter / q, jitter / q, pts.shape)
    return pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy()


def monos3(m):
    return [(a, b, d - a - b) for d in range(m + 1) for a in range(d, -1, -1)
            for b in range(d - a, -1, -1)]


@pytest.mark.parametrize("k", [1, 10, 20, 35])
def test_knn3_matches_kdtree(k):
    x, y, z = jittered_cube(9, seed=3)
    nb = oracle.knn3(x, y, z, k)
    pts = np.stack([x, y, z], 1)
    dist, _ = cKDTree(pts).query(pts, k=k)
    dist = dist.reshape(len(x), k)
    d_or = np.sqrt(((pts[nb] - pts[:, None, :]) ** 2).sum(-1))
    assert np.allclose(np.sort(d_or, 1), dist, rtol=1e-14, atol=0)
    assert np.all(nb[:, 0] == np.arange(len(x)))          # self first
    for i in range(0, len(x), 37):
        inside = set(np.nonzero(np.linalg.norm(pts - pts[i], axis=1) < dist[i, -1] * (1 - 1e-12))[0])
        assert inside <= set(nb[i].tolist())


def test_knn3_ties_python_sort():
    g = np.arange(4, dtype=np.float64)
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    x[5], y[5], z[5] = x[9], y[9], z[9]     # a duplicate node
    x[11] = np.nan                          # never selected
    rng = np.random.default_rng(0)
    perm = rng.permutation(len(x))
    x, y, z = x[perm], y[perm], z[perm]
    k = 19
    nb = oracle.knn3(x, y, z, k)
    for i in range(len(x)):
        keys = []
        for j in range(len(x)):
            dx, dy, dz = x[j] - x[i], y[j] - y[i], z[j] - z[i]
            d2 = (dx * dx + dy * dy) + dz * dz
            if d2 == d2:
                keys.append((d2, j))
        keys.sort()
        want = [j for _, j in keys[:k]] + [-1] * max(0, k - len(keys))
        assert nb[i].tolist() == want, i


@pytest.mark.parametrize("m,n", [(2, 20), (3, 30), (4, 45), (4, 70)])
def test_weights3_reproduce_polynomials(m, n):
    x, y, z = jittered_cube(8, seed=5)
    nb = oracle.knn3(x, y, z, n)
    rows = np.arange(0, len(x), 23)
    w, st = oracle.weights3(x, y, z, nb, m, n, rows=rows)
    assert np.all(st == oracle.OK)
    for t, i in enumerate(rows):
        idx = nb[i]
        dx, dy, dz = x[idx] - x[i], y[idx] - y[i], z[idx] - z[i]
        for a, b, c in monos3(m):
            f = dx ** a * dy ** b * dz ** c
            want = 2.0 if sorted((a, b, c)) == [0, 0, 2] else 0.0
            got = np.dot(w[t], f)
            scale = np.abs(w[t] * f).sum() + want
            assert abs(got - want) <= 1e-10 * scale, (i, (a, b, c), got)
    # one degree higher is not reproduced (the set is exactly degree <= m):
    # lap x^(m+1) vanishes at the centre, the weights do not annihilate it
    i = rows[3]
    f = (x[nb[i]] - x[i]) ** (m + 1)
    assert abs(np.dot(w[3], f)) > 1e-6 * np.abs(w[3] * f).sum()


@pytest.mark.parametrize("m", [2, 3, 4])
def test_weights3_laplacian_of_phs_interpolant(m):
    import mpmath
    n = {2: 20, 3: 30, 4: 70}[m]
    x, y, z = jittered_cube(7, seed=9)
    nb = oracle.knn3(x, y, z, n)
    rng = np.random.default_rng(8)
    ex = monos3(m)
    for i in [40, 171]:
        idx = nb[i]
        w, st = oracle.weights3(x, y, z, nb, m, n, rows=[i])
        assert st[0] == 0
        px, py, pz = x[idx], y[idx], z[idx]
        cx, cy, cz = x[i], y[i], z[i]
        f = rng.standard_normal(n)
        A = np.sqrt((px[:, None] - px[None]) ** 2 + (py[:, None] - py[None]) ** 2 +
                    (pz[:, None] - pz[None]) ** 2) ** 3
        P = np.array([[(a_ - cx) ** e[0] * (b_ - cy) ** e[1] * (c_ - cz) ** e[2] for e in ex]
                      for a_, b_, c_ in zip(px, py, pz)])
        M = np.block([[A, P], [P.T, np.zeros((len(ex), len(ex)))]])
        coef = np.linalg.solve(M, np.concatenate([f, np.zeros(len(ex))]))
        with mpmath.workdps(30):
            def s_f(X, Y, Z):
                acc = mpmath.mpf(0)
                for k in range(n):
                    acc += coef[k] * mpmath.sqrt((X - px[k]) ** 2 + (Y - py[k]) ** 2 +
                                                 (Z - pz[k]) ** 2) ** 3
                for j, e in enumerate(ex):
                    acc += coef[n + j] * (X - cx) ** e[0] * (Y - cy) ** e[1] * (Z - cz) ** e[2]
                return acc
            X0, Y0, Z0 = mpmath.mpf(cx), mpmath.mpf(cy), mpmath.mpf(cz)
            lap = mpmath.diff(lambda t: s_f(t, Y0, Z0), X0, 2) + \
                mpmath.diff(lambda t: s_f(X0, t, Z0), Y0, 2) + \
                mpmath.diff(lambda t: s_f(X0, Y0, t), Z0, 2)
        got = float(np.dot(w[0, :n], f))
        assert abs(got - float(lap)) <= 1e-8 * np.abs(w[0, :n] * f).sum(), (got, float(lap))


def test_weights3_scale_and_rigid_motion():
    x, y, z = jittered_cube(7, seed=12)
    nb = oracle.knn3(x, y, z, 20)
    rows = np.arange(0, len(x), 11)
    w, st = oracle.weights3(x, y, z, nb, 2, 20, rows=rows)
    assert np.all(st == 0)
    a = 0.37
    w2, _ = oracle.weights3(a * x, a * y, a * z, nb, 2, 20, rows=rows)
    assert np.allclose(w2 * a * a, w, rtol=1e-9, atol=1e-9 * np.abs(w).max())
    th = np.random.default_rng(4).standard_normal((3, 3))
    Q, _ = np.linalg.qr(th)
    pts = np.stack([x, y, z], 1) @ Q.T + np.array([3.0, -1.0, 0.5])
    w3, _ = oracle.weights3(pts[:, 0].copy(), pts[:, 1].copy(), pts[:, 2].copy(), nb, 2, 20,
                            rows=rows)
    assert np.allclose(w3, w, rtol=1e-8, atol=1e-8 * np.abs(w).max())
    assert np.abs(w.sum(1)).max() <= 1e-9 * np.abs(w).max()


def test_weights3_status_codes():
    x, y, z = jittered_cube(5, seed=2)
    nb = oracle.knn3(x, y, z, 20)
    nb[3, 4] = nb[3, 2]               # duplicate support node
    nb[4, 7] = len(x) + 1             # index out of range
    xx = x.copy()
    xx[nb[6, 5]] = np.inf             # non-finite coordinate
    w, st = oracle.weights3(xx, y, z, nb, 2, 20)
    assert st[3] == oracle.DUPLICATE and st[4] == oracle.BAD_INDEX and st[6] == oracle.NONFINITE
    assert np.all(np.isnan(w[[3, 4, 6]]))
    # a coplanar support: the z column of P vanishes -> a zero pivot
    g = np.arange(6, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    xp, yp, zp = X.ravel().copy(), Y.ravel().copy(), np.zeros(36)
    nbp = oracle.knn3(xp, yp, zp, 20)
    w, st = oracle.weights3(xp, yp, zp, nbp, 2, 20)
    assert np.all(st == oracle.SINGULAR)


# ---- first derivatives in three dimensions (oracle.weights3_op) -----------

D3 = [(oracle.D3_DX, (1, 0, 0)), (oracle.D3_DY, (0, 1, 0)), (oracle.D3_DZ, (0, 0, 1))]


@pytest.mark.parametrize("op,axis", D3)
@pytest.mark.parametrize("m,n", [(2, 20), (3, 30), (4, 70)])
def test_weights3_derivative_reproduce_polynomials(op, axis, m, n):
    x, y, z = jittered_cube(8, seed=15)
    nb = oracle.knn3(x, y, z, n)
    rows = np.arange(0, len(x), 29)
    w, st = oracle.weights3_op(x, y, z, nb, m, n, op, rows=rows)
    assert np.all(st == oracle.OK)
    for t, i in enumerate(rows):
        idx = nb[i]
        dx, dy, dz = x[idx] - x[i], y[idx] - y[i], z[idx] - z[i]
        for e in monos3(m):
            f = dx ** e[0] * dy ** e[1] * dz ** e[2]
            want = 1.0 if e == axis else 0.0
            got = np.dot(w[t], f)
            assert abs(got - want) <= 1e-10 * (np.abs(w[t] * f).sum() + want), (i, e, got)


def test_weights3_derivative_of_phs_interpolant():
    """w . f equals the derivative of the r^3 + monomial interpolant of f at
    the centre (30-digit numerical differentiation): pins -3 r u_axis, its
    sign and its component, which polynomial reproduction cannot see."""
    import mpmath
    m, n = 2, 20
    x, y, z = jittered_cube(7, seed=19)
    nb = oracle.knn3(x, y, z, n)
    rng = np.random.default_rng(18)
    ex = monos3(m)
    for i in [57, 200]:
        idx = nb[i]
        px, py, pz = x[idx], y[idx], z[idx]
        cx, cy, cz = x[i], y[i], z[i]
        f = rng.standard_normal(n)
        A = np.sqrt((px[:, None] - px[None]) ** 2 + (py[:, None] - py[None]) ** 2 +
                    (pz[:, None] - pz[None]) ** 2) ** 3
        P = np.array([[(a_ - cx) ** e[0] * (b_ - cy) ** e[1] * (c_ - cz) ** e[2] for e in ex]
                      for a_, b_, c_ in zip(px, py, pz)])
        M = np.block([[A, P], [P.T, np.zeros((len(ex), len(ex)))]])
        coef = np.linalg.solve(M, np.concatenate([f, np.zeros(len(ex))]))
        with mpmath.workdps(30):
            def s_f(X, Y, Z):
                acc = mpmath.mpf(0)
                for k in range(n):
                    acc += coef[k] * mpmath.sqrt((X - px[k]) ** 2 + (Y - py[k]) ** 2 +
                                                 (Z - pz[k]) ** 2) ** 3
                for j, e in enumerate(ex):
                    acc += coef[n + j] * (X - cx) ** e[0] * (Y - cy) ** e[1] * (Z - cz) ** e[2]
                return acc
            X0, Y0, Z0 = mpmath.mpf(cx), mpmath.mpf(cy), mpmath.mpf(cz)
            want = {oracle.D3_DX: float(mpmath.diff(lambda t: s_f(t, Y0, Z0), X0, 1)),
                    oracle.D3_DY: float(mpmath.diff(lambda t: s_f(X0, t, Z0), Y0, 1)),
                    oracle.D3_DZ: float(mpmath.diff(lambda t: s_f(X0, Y0, t), Z0, 1))}
        for op, _ in D3:
            w, st = oracle.weights3_op(x, y, z, nb, m, n, op, rows=[i])
            assert st[0] == 0
            got = float(np.dot(w[0, :n], f))
            assert abs(got - want[op]) <= 1e-8 * np.abs(w[0, :n] * f).sum(), (op, got, want[op])


def test_weights3_derivative_scale_and_laplacian_op():
    x, y, z = jittered_cube(6, seed=13)
    nb = oracle.knn3(x, y, z, 20)
    w, _ = oracle.weights3_op(x, y, z, nb, 2, 20, oracle.D3_DZ)
    a = 2.5
    w2, _ = oracle.weights3_op(a * x, a * y, a * z, nb, 2, 20, oracle.D3_DZ)
    assert np.allclose(w2 * a, w, rtol=1e-9, atol=1e-9 * np.abs(w).max())
    w0, st0 = oracle.weights3_op(x, y, z, nb, 2, 20, 0)
    wl, stl = oracle.weights3(x, y, z, nb, 2, 20)
    assert np.array_equal(w0, wl, equal_nan=True) and np.array_equal(st0, stl)
