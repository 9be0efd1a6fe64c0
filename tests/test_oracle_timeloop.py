"""Pins for the oracle's explicit pseudo-time loop (section IV, eq. (3)).

* one step against exact rational arithmetic of u + dt (f + sum_k w u);
* many steps against an independent SciPy sparse iteration;
* the discrete steady state (SciPy spsolve of W u = -f with the Dirichlet
  values) is a fixed point; boundary values never change;
* the iteration contracts toward that steady state.
"""

from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from paper_2107_03632_amd import nodes


def _setup(nx=14, m=2, n=12, seed=6):
    ns = nodes.unit_square(nx, seed=seed)
    nbr = oracle.knn(ns.x, ns.y, n)
    w, st = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    assert np.all(st == 0)
    u_exact, F = nodes.manufactured(ns.x, ns.y)
    f = -F  # the pseudo-time form of eq. (3): du/dt = lap u + f
    u0 = np.where(ns.is_boundary != 0, u_exact, 0.0)
    return ns, nbr, w, f, u0, u_exact


def _csr(ns, nbr, w, n):
    N = ns.n_nodes
    rows = np.repeat(np.arange(N), n)
    W = sp.csr_matrix((w[:, :n].ravel(), (rows, nbr[:, :n].ravel())), shape=(N, N))
    return W


def test_one_step_matches_exact_arithmetic():
    ns, nbr, w, f, u0, _ = _setup()
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal(ns.n_nodes)
    dt = 1e-3
    u1 = oracle.time_steps(nbr, w, 12, f, u0, dt, 1, is_boundary=ns.is_boundary)
    eps = np.finfo(float).eps
    for i in range(ns.n_nodes):
        if ns.is_boundary[i]:
            assert u1[i] == u0[i]
            continue
        lap = sum(Fraction(w[i, k]) * Fraction(u0[nbr[i, k]]) for k in range(12))
        exact = Fraction(u0[i]) + Fraction(dt) * (Fraction(f[i]) + lap)
        scale = abs(u0[i]) + dt * (abs(f[i]) + sum(abs(w[i, k] * u0[nbr[i, k]]) for k in range(12)))
        assert abs(u1[i] - float(exact)) <= 8 * eps * scale, i


def test_many_steps_match_scipy_iteration():
    ns, nbr, w, f, u0, _ = _setup()
    W = _csr(ns, nbr, w, 12)
    inter = ns.is_boundary == 0
    dt, steps = 1e-4, 50
    u = u0.copy()
    for _ in range(steps):
        un = u + dt * (f + W @ u)
        u = np.where(inter, un, u)
    uo = oracle.time_steps(nbr, w, 12, f, u0, dt, steps, is_boundary=ns.is_boundary)
    assert np.abs(uo - u).max() <= 1e-12 * max(1.0, np.abs(u).max())
    assert np.array_equal(uo[~inter], u0[~inter])


def test_steady_state_is_a_fixed_point_and_iteration_contracts():
    ns, nbr, w, f, u0, u_exact = _setup()
    W = _csr(ns, nbr, w, 12).tolil()
    rhs = -f.copy()
    for i in np.nonzero(ns.is_boundary)[0]:
        W.rows[i] = [i]
        W.data[i] = [1.0]
        rhs[i] = u_exact[i]
    ustar = spla.spsolve(W.tocsr(), rhs)
    dt = 1e-4
    us = oracle.time_steps(nbr, w, 12, f, ustar, dt, 20, is_boundary=ns.is_boundary)
    assert np.abs(us - ustar).max() <= 1e-10
    # contraction toward the steady state from zero interior values
    e0 = np.abs(u0 - ustar).max()
    e1 = np.abs(oracle.time_steps(nbr, w, 12, f, u0, dt, 200, is_boundary=ns.is_boundary) - ustar).max()
    e2 = np.abs(oracle.time_steps(nbr, w, 12, f, u0, dt, 2000, is_boundary=ns.is_boundary) - ustar).max()
    assert e2 < e1 < e0
    # the discrete steady state approximates the closed form (m = 2 at
    # h = 1/15: discretisation error of order h^2)
    assert np.abs(ustar - u_exact).max() < 5e-2


def test_bad_index_gives_nan_and_argument_errors():
    ns, nbr, w, f, u0, _ = _setup()
    nb = nbr.copy()
    i = int(np.nonzero(ns.is_boundary == 0)[0][3])
    nb[i, 5] = ns.n_nodes + 7
    u = oracle.time_steps(nb, w, 12, f, u0, 1e-4, 1, is_boundary=ns.is_boundary)
    assert np.isnan(u[i]) and np.isfinite(np.delete(u, i)).all()
    with pytest.raises(ValueError):
        oracle.time_steps(nbr, w, 0, f, u0, 1e-4, 1)
    with pytest.raises(ValueError):
        oracle.time_steps(nbr, w, 13, f, u0, 1e-4, 1)
