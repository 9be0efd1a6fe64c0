"""Pin for the whole oracle path: the steady Dirichlet Poisson problem of
section IV (lap u = f, u = sin(pi x) sin(pi y)) solved with the oracle's CSR
operator converges at order ~m as h shrinks (the approximation order of PHS +
monomials of degree m, sections I and V)."""

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spl

import oracle
from paper_2107_03632_amd import nodes

NFM = {2: 12, 4: 30, 6: 56}


def _solve_error(cells, m):
    ns = nodes.unit_square(cells, seed=10 + cells)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w, st = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    assert np.all(st == 0)
    rp, c, v = oracle.csr(nbr, w, n=n, is_boundary=ns.is_boundary)
    A = sp.csr_matrix((v, c, rp), shape=(ns.n_nodes, ns.n_nodes))
    ue, f = nodes.manufactured(ns.x, ns.y)
    b = np.where(ns.is_boundary == 1, ue, f)
    u = oracle.solve(rp, c, v, b)
    # the solve itself: a small residual, and SciPy's solver called directly
    assert np.abs(A @ u - b).max() <= 1e-9 * np.abs(b).max()
    assert np.array_equal(u, spl.spsolve(A.tocsc(), b))
    return np.abs(u - ue).max()


@pytest.mark.parametrize("m", [2, 4, 6])
def test_convergence_order(m):
    cells = [16, 24, 32, 48]
    errs = [_solve_error(c, m) for c in cells]
    slope = np.polyfit(np.log(1.0 / np.array(cells)), np.log(errs), 1)[0]
    assert slope >= m - 0.5, (slope, errs)
    assert errs[-1] < errs[0]
