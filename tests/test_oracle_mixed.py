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
    assert stm[0] == oracle.FELL_BACK and 1 <= it[0] <= 10
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


def test_lu32_is_a_partial_pivoting_factorisation():
    # P M32 = L U to FP32 rounding, unit L, and every pivot the first largest
    # |entry| of its column among the rows not yet pivoted
    ns = nodes.unit_square(12, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 30)
    st, M, rhs, s = oracle.assemble(ns.x, ns.y, 77, nbr[77], 4)
    st, LU, perm, dinv = oracle.lu32(M)
    assert st == oracle.OK
    K = M.shape[0]
    A = M.astype(np.float32).astype(np.float64)
    L = np.tril(LU.astype(np.float64), -1) + np.eye(K)
    U = np.triu(LU.astype(np.float64))
    PA = A.copy()
    for c in range(K):
        p = perm[c]
        PA[[c, p]] = PA[[p, c]]
    assert np.abs(PA - L @ U).max() <= 64 * np.finfo(np.float32).eps * np.abs(A).max()
    assert np.abs(L).max() <= 1.0
    assert np.allclose(dinv.astype(np.float64), 1.0 / np.diag(U), rtol=1e-7)


# The refinement's fallback rule (a correction larger than half the previous
# one, the first compared with max|z0|) and its cap of 10 corrections are
# pinned by stencils whose FP32 factors contract the error at a known rate.
# The rate comes from the oracle's FP32 factors F = P^T L U, iterated here in
# FP64 arithmetic: z0 = F^-1 b, then z += F^-1 (b - M z).  Two support nodes
# are pulled together by delta to set cond(M), hence the rate.

def _perturbed(i, k):
    ns = nodes.unit_square(12, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 12)
    d = 10.0 ** (-4.0 - k / 20.0)
    x, y = ns.x.copy(), ns.y.copy()
    x[nbr[i, 4]] = x[nbr[i, 3]] + d
    y[nbr[i, 4]] = y[nbr[i, 3]] + 0.3 * d
    return x, y, nbr


def _model_ratios(M, b, steps=10):
    st, LU, perm, _ = oracle.lu32(M)
    assert st == oracle.OK
    K = M.shape[0]
    L = np.tril(LU.astype(np.float64), -1) + np.eye(K)
    U = np.triu(LU.astype(np.float64))
    P = np.eye(K)
    for c in range(K):
        p = perm[c]
        P[[c, p]] = P[[p, c]]
    F = P.T @ L @ U
    z = np.linalg.solve(F, b)
    prev = np.abs(z).max()
    out = []
    for _ in range(steps):
        d = np.linalg.solve(F, b - M @ z)
        z = z + d
        dn = np.abs(d).max()
        out.append(dn / prev)
        prev = dn
    return np.array(out)


@pytest.mark.parametrize("i,k,lo,hi,tries", [
    (40, 16, 0.70, 0.80, 1),   # corrections shrink by ~0.75: the first one already
    (90, 12, 0.78, 0.82, 1),   # exceeds half of max|z0|
    (90, 7, 0.50, 0.52, 1),    # just above one half
    (40, 8, 0.47, 0.50, 10),   # just below one half: refined until the cap
    (90, 1, 0.20, 0.22, 10),   # ~0.2 per step: too slow for 1e-12 in 10
    (77, 9, 0.32, 0.34, 10),
])
def test_mixed_fallback_rule_and_cap(i, k, lo, hi, tries):
    x, y, nbr = _perturbed(i, k)
    st, M, rhs, s = oracle.assemble(x, y, i, nbr[i], 2)
    rat = _model_ratios(M, rhs)
    assert np.all((rat >= lo) & (rat <= hi)), rat
    wm, stm, it = oracle.weights_mixed(x, y, nbr, m=2, n=12, rows=[i])
    w64, st64 = oracle.weights(x, y, nbr, m=2, n=12, rows=[i])
    assert st64[0] == oracle.OK
    assert stm[0] == oracle.FELL_BACK
    assert it[0] == tries
    assert np.array_equal(wm, w64)


# ---- the second reading: the FP32 factorisation as a Gauss-Jordan inverse ----

def test_gj32_inverts_the_fp32_matrix():
    # S = (P M32)^-1 to FP32 accuracy, S (P M32) = I, with M32 = (float) M
    ns = nodes.unit_square(12, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 30)
    st, M, rhs, s = oracle.assemble(ns.x, ns.y, 77, nbr[77], 4)
    st, S, perm = oracle.gj32(M)
    assert st == oracle.OK
    K = M.shape[0]
    A = M.astype(np.float32).astype(np.float64)
    PA = A.copy()
    for c in range(K):
        p = perm[c]
        PA[[c, p]] = PA[[p, c]]
    S = S.astype(np.float64)
    cond = np.linalg.cond(PA, np.inf)
    eps = np.finfo(np.float32).eps
    assert np.abs(S @ PA - np.eye(K)).max() <= K * cond * eps
    inv = np.linalg.inv(PA)
    assert np.abs(S - inv).max() <= K * cond * eps * np.abs(inv).max()
    # the pivots are those of partial pivoting: the same rows as the LU
    # factorisation picks on this well-conditioned system
    st2, LU, perm_lu, _ = oracle.lu32(M)
    assert np.array_equal(perm, perm_lu)


def test_gj32_small_cases_by_hand():
    # [[1, 2, 0], [2, 1, 1], [0, 1, 2]]: column 0 pivots on row 1 (|2| > |1|),
    # then the inverse of the swapped matrix is (P M)^-1 = M^-1 P^T, det M = -7
    M = np.array([[1.0, 2.0, 0.0], [2.0, 1.0, 1.0], [0.0, 1.0, 2.0]])
    st, S, perm = oracle.gj32(M)
    assert st == oracle.OK and perm[0] == 1
    P = np.eye(3)
    P[[0, 1]] = P[[1, 0]]
    exact = np.array([[1.0, -4.0, 2.0], [-4.0, 2.0, -1.0], [2.0, -1.0, -3.0]]) / -7.0
    assert np.allclose(S.astype(np.float64), exact @ P.T, rtol=0, atol=1e-6)
    # a tie in |entry|: the first of the equal rows is the pivot (no swap)
    st, S, perm = oracle.gj32(np.array([[1.0, 1.0], [-1.0, 1.0]]))
    assert st == oracle.OK and perm[0] == 0
    assert np.allclose(S, np.array([[0.5, -0.5], [0.5, 0.5]]), rtol=0, atol=0)
    # a zero column: singular
    st, S, perm = oracle.gj32(np.array([[0.0, 1.0], [0.0, 2.0]]))
    assert st == oracle.SINGULAR


@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_gj_matches_fp64_and_exact_solution(m):
    ns = nodes.unit_disk(2000, 160, seed=31)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w64, st64 = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    wm, stm, it = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n, form=oracle.MIXED_GJ)
    assert np.all((stm == 0) | (stm == oracle.FELL_BACK))
    e = np.abs(wm - w64).max(axis=1) / np.abs(w64).max(axis=1)
    assert e.max() <= 1e-9
    assert np.all(it[stm == 0] >= 1) and np.all(it <= 10)
    for i in [0, 411, ns.n_nodes - 3]:
        st, M, rhs, s = oracle.assemble(ns.x, ns.y, i, nbr[i], m)
        with mpmath.workdps(50):
            zm = mpmath.lu_solve(mpmath.matrix(M.tolist()), mpmath.matrix(rhs.tolist()))
            w_ex = np.array([float(zm[k] / (mpmath.mpf(s) ** 2)) for k in range(n)])
        assert np.abs(wm[i, :n] - w_ex).max() / np.abs(w_ex).max() <= 1e-9


def _model_ratios_gj(M, b, steps=10):
    # the oracle's FP32 inverse S = (P M32)^-1, iterated in FP64:
    # z0 = S P b, z += S P (b - M z)
    st, S, perm = oracle.gj32(M)
    assert st == oracle.OK
    K = M.shape[0]
    P = np.eye(K)
    for c in range(K):
        p = perm[c]
        P[[c, p]] = P[[p, c]]
    F = S.astype(np.float64) @ P
    z = F @ b
    prev = np.abs(z).max()
    out = []
    for _ in range(steps):
        d = F @ (b - M @ z)
        z = z + d
        dn = np.abs(d).max()
        out.append(dn / prev)
        prev = dn
    return np.array(out)


@pytest.mark.parametrize("i,k,lo,hi,tries", [
    (90, 4, 0.53, 0.58, 1),    # corrections shrink by ~0.57: above one half at once
    (90, 7, 2.2, 2.5, 1),      # they grow
    (90, 12, 0.42, 0.46, 10),  # below one half: refined until the cap
    (90, 1, 0.22, 0.24, 10),   # ~0.23 per step: too slow for 1e-12 in 10
])
def test_mixed_gj_fallback_rule_and_cap(i, k, lo, hi, tries):
    x, y, nbr = _perturbed(i, k)
    st, M, rhs, s = oracle.assemble(x, y, i, nbr[i], 2)
    rat = _model_ratios_gj(M, rhs)
    assert np.all((rat >= lo) & (rat <= hi)), rat
    wm, stm, it = oracle.weights_mixed(x, y, nbr, m=2, n=12, rows=[i], form=oracle.MIXED_GJ)
    w64, st64 = oracle.weights(x, y, nbr, m=2, n=12, rows=[i])
    assert st64[0] == oracle.OK
    assert stm[0] == oracle.FELL_BACK
    assert it[0] == tries
    assert np.array_equal(wm, w64)


@pytest.mark.parametrize("form", [oracle.MIXED_LU, oracle.MIXED_GJ])
@pytest.mark.parametrize("m", [2, 4, 6])
@pytest.mark.parametrize("op", [oracle.D_DX, oracle.D_DY])
def test_mixed_derivative_weights(op, m, form):
    """The mixed form of the derivative operators: the same refinement and
    fallback rule on the operator's right-hand side.  The refined weights
    agree with the FP64 derivative weights to the 1e-9 target, a stencil
    that fell back carries exactly the FP64 weights, and the weights
    differentiate every monomial of degree <= m exactly at the centre (the
    polynomial part of eq. (1) with L = d/dx or d/dy)."""
    ns = nodes.unit_disk(1500, 140, seed=34)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w64, st64 = oracle.weights_op(ns.x, ns.y, nbr, m, n, op)
    wm, stm, it = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n, form=form, op=op)
    assert np.all(st64 == 0)
    assert np.all((stm == 0) | (stm == oracle.FELL_BACK))
    e = np.abs(wm - w64).max(axis=1) / np.abs(w64).max(axis=1)
    assert e.max() <= 1e-9
    assert np.all(it[stm == 0] >= 1) and np.all(it <= 10)
    fb = stm == oracle.FELL_BACK
    assert np.array_equal(wm[fb], w64[fb])
    dx = ns.x[nbr] - ns.x[:, None]
    dy = ns.y[nbr] - ns.y[:, None]
    for a in range(m + 1):
        for b in range(m + 1 - a):
            p = dx ** a * dy ** b
            want = 1.0 if (a, b) == ((1, 0) if op == oracle.D_DX else (0, 1)) else 0.0
            got = (wm * p).sum(axis=1)
            scale = np.abs(wm * p).sum(axis=1) + want
            assert np.max(np.abs(got - want) / scale) < 1e-9, (a, b)


def test_mixed_laplacian_through_the_operator_entry():
    ns = nodes.unit_disk(800, 100, seed=35)
    nbr = oracle.knn(ns.x, ns.y, 30)
    a = oracle.weights_mixed(ns.x, ns.y, nbr, m=4, n=30)
    b = oracle.weights_mixed(ns.x, ns.y, nbr, m=4, n=30, op=oracle.LAPLACIAN)
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
