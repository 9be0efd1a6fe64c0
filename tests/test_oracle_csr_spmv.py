"""Pins for the oracle's CSR operator (eq. (1) rows, Dirichlet identity rows
of section IV) and its SpMV (eq. (3) uses W u), against SciPy."""

import numpy as np
import scipy.sparse as sp

import oracle
from paper_2107_03632_amd import nodes


def test_csr_matches_scipy_and_spmv():
    ns = nodes.unit_disk(2000, 150, seed=4)
    n = 30
    nbr = oracle.knn(ns.x, ns.y, n)
    w, st = oracle.weights(ns.x, ns.y, nbr, m=4, n=n)
    assert np.all(st == 0)
    rp, col, val = oracle.csr(nbr, w, n=n, is_boundary=ns.is_boundary)
    rows = np.repeat(np.arange(ns.n_nodes), n)
    keep = ns.is_boundary[rows] == 0
    r = np.concatenate([rows[keep], np.nonzero(ns.is_boundary)[0]])
    c = np.concatenate([nbr.ravel()[keep], np.nonzero(ns.is_boundary)[0]])
    v = np.concatenate([w.ravel()[keep], np.ones(int(ns.is_boundary.sum()))])
    ref = sp.csr_matrix((v, (r, c)), shape=(ns.n_nodes, ns.n_nodes))
    ref.sort_indices()
    assert np.array_equal(rp, ref.indptr)
    assert np.array_equal(col, ref.indices)
    assert np.array_equal(val, ref.data)
    u, f = nodes.manufactured(ns.x, ns.y)
    y = oracle.spmv(rp, col, val, u, f)
    y_ref = ref @ u - f
    scale = np.abs(ref).dot(np.abs(u)) + np.abs(f)
    assert np.all(np.abs(y - y_ref) <= 1e-13 * scale)
    # residual of the manufactured solution is the consistency error: small
    # relative to |f| on interior rows
    inter = ns.is_boundary == 0
    assert np.abs(y[inter]).max() < 1e-2 * np.abs(f).max()


def test_csr_orders_columns_and_keeps_duplicates():
    nbr = np.array([[3, 1, 2, 1], [0, 2, 1, 3]], dtype=np.int32)
    w = np.array([[10., 11., 12., 13.], [1., 2., 3., 4.]])
    rp, col, val = oracle.csr(nbr, w, n=4, is_boundary=np.array([0, 1], np.uint8))
    assert list(rp) == [0, 4, 5]
    assert list(col) == [1, 1, 2, 3, 1]
    assert list(val) == [11., 13., 12., 10., 1.]
