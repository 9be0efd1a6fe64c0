"""Pins for the oracle's mixed-precision weights (FP32 factorisation of the
FP64-assembled system + FP64 iterative refinement, FP64 fallback).

The refined weights must agree with the exactly solved system (50-digit
solve of the same FP64 matrix) and with the FP64 oracle to the 1e-9 target;
a stencil whose FP32 factorisation cannot be refined must come back with
status FELL_BACK and exactly the FP64 weights.
"""

import mpmath
import numpy as np
import pytest

import oracle
from paper_2107_03632_amd import nodes

NFM = {2: 12, 4: 30, 6: 56}


@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_matches_fp64_oracle(m):
    ns = nodes.unit_disk(2000, 160, seed=31)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w64, st64 = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    wm, stm, it = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n)
    assert np.all(st64 == 0)
    assert np.all((stm == 0) | (stm == oracle.FELL_BACK))
    e = np.abs(wm - w64).max(axis=1) / np.abs(w64).max(axis=1)
    assert e.max() <= 1e-9
    assert np.all(it[stm == 0] >= 1) and np.all(it <= 10)
    fb = stm == oracle.FELL_BACK
    assert np.array_equal(wm[fb], w64[fb])


@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_matches_exact_solution(m):
    ns = nodes.unit_disk(2000, 160, seed=31)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    for i in [0, 411, ns.n_nodes - 3]:
        st, M, rhs, s = oracle.assemble(ns.x, ns.y, i, nbr[i], m)
        wm, stm, _ = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n, rows=[i])
        with mpmath.workdps(50):
            zm = mpmath.lu_solve(mpmath.matrix(M.tolist()), mpmath.matrix(rhs.tolist()))
            w_ex = np.array([float(zm[k] / (mpmath.mpf(s) ** 2)) for k in range(n)])
        assert np.abs(wm[0, :n] - w_ex).max() / np.abs(w_ex).max() <= 1e-9


def test_mixed_falls_back_to_fp64_on_ill_conditioned_stencil():
    # two support nodes 1e-4 apart: cond(M) ~ 1e8, beyond what FP32 factors
    # can refine, while the FP64 factorisation still succeeds
    ns = nodes.unit_square(8, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 12)
    i = 30
    x, y = ns.x.copy(), ns.y.copy()
    x[nbr[i, 4]] = x[nbr[i, 3]] + 1e-4
    y[nbr[i, 4]] = y[nbr[i, 3]]
    w64, st64 = oracle.weights(x, y, nbr, m=2, n=12, rows=[i])
    wm, stm, it = oracle.weights_mixed(x, y, nbr, m=2, n=12, rows=[i])
    assert st64[0] == oracle.OK
    assert stm[0] == oracle.FELL_BACK and it[0] == 0
    assert np.array_equal(wm, w64)
    # a milder pair (1e-3 apart) is refined instead, to the same weights
    x[nbr[i, 4]] = x[nbr[i, 3]] + 1e-3
    w64, _ = oracle.weights(x, y, nbr, m=2, n=12, rows=[i])
    wm, stm, it = oracle.weights_mixed(x, y, nbr, m=2, n=12, rows=[i])
    assert stm[0] == oracle.OK and it[0] >= 3
    assert np.abs(wm - w64).max() / np.abs(w64).max() <= 1e-9


def test_mixed_reports_assembly_failures_without_fallback():
    ns = nodes.unit_square(8, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 12)
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]
    wm, stm, _ = oracle.weights_mixed(ns.x, ns.y, nb, m=2, n=12, rows=[10, 11])
    assert stm[0] == oracle.DUPLICATE and np.all(np.isnan(wm[0]))
    assert stm[1] == oracle.OK
