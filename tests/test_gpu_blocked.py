"""Weights from the blocked kernels whose trailing updates run on the matrix
cores (K = 84: m = 6, n = 56, two wavefronts per stencil; K = 45: m = 4,
n = 30, one wavefront per stencil), against the oracle and against the
unblocked kernels (the path taken when the factors are saved for the
adjoint).

The blocked elimination applies to every entry the same fused updates, in
the same order, as the unblocked one, so the bar here is stricter than the
1e-11 of the general parity tests: every weight is the same double (NaN
where the stencil failed), and every status is the same.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu

ORDERS = [(4, 30), (6, 56)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


def both_paths(x, y, nbr, m, n):
    X, Y, NB = dev(x), dev(y), dev(nbr)
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=m, n=n)              # blocked, MFMA
    w2, st2, _ = rb.rbffd_weights(X, Y, NB, m=m, n=n, save=True)  # unblocked
    return host(w), host(st), host(w2), host(st2)


def check_same(x, y, nbr, m, n, label):
    w_ref, st_ref = oracle.weights(x, y, nbr, m=m, n=n)
    w, st, w2, st2 = both_paths(x, y, nbr, m, n)
    say(label, f"m={m}", "stencils", nbr.shape[0], "statuses", np.bincount(st_ref))
    assert np.array_equal(st, st_ref)
    assert np.array_equal(st2, st_ref)
    assert np.array_equal(w, w2, equal_nan=True)
    ok = st_ref == 0
    assert np.array_equal(w[ok], w_ref[ok])
    assert np.all(np.isnan(w[~ok]))
    assert np.all(w[ok][:, n:] == 0.0)


@pytest.mark.parametrize("m,n", ORDERS)
def test_blocked_disk_bit_exact(m, n):
    ns = nodes.unit_disk(3000, 200, seed=21)
    nbr = oracle.knn(ns.x, ns.y, 64)
    check_same(ns.x, ns.y, np.ascontiguousarray(nbr[:, :n]), m, n, f"disk 3200, k_stride {n}")
    # a wider row stride (zeros past n)
    check_same(ns.x, ns.y, nbr, m, n, "disk 3200, k_stride 64")


@pytest.mark.parametrize("m,n", ORDERS)
def test_blocked_exact_lattice_ties(m, n):
    # an unjittered lattice: many entries of equal magnitude, so the pivot
    # search takes its exact (|a|, position) path often
    ns = nodes.cell_centred_square(24, seed=7, jitter=0.0)
    nbr = oracle.knn(ns.x, ns.y, n)
    check_same(ns.x, ns.y, nbr, m, n, "exact lattice 24x24")


@pytest.mark.parametrize("m,n", ORDERS)
def test_blocked_status_codes(m, n):
    ns = nodes.unit_square(12, seed=3)
    x, y = ns.x.copy(), ns.y.copy()
    nbr = oracle.knn(x, y, n)
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]            # duplicate support node
    nb[11, n // 2] = x.size + 4      # out of range
    nb[12, n - 1] = -1
    xx = x.copy()
    xx[nbr[13, n - 3]] = np.inf      # non-finite coordinate
    check_same(xx, y, nb, m, n, "status codes")
    # collinear support: the P block is rank deficient -> zero pivot
    xl = np.linspace(0.0, 1.0, n + 4)
    yl = np.full(n + 4, 0.25)
    nl = np.tile(np.arange(n, dtype=np.int32), (n + 4, 1))
    w_ref, st_ref = oracle.weights(xl, yl, nl, m=m, n=n)
    assert np.all(st_ref == oracle.SINGULAR)
    w, st, w2, st2 = both_paths(xl, yl, nl, m, n)
    assert np.array_equal(st, st_ref) and np.array_equal(st2, st_ref)
    assert np.all(np.isnan(w))


@pytest.mark.parametrize("m,n,workload", [(4, 30, "disk_100k_m4"), (6, 56, "square_1m_m6")])
def test_blocked_full_size_sampled(m, n, workload):
    # the full workloads, in the launch the benchmark times
    ns = nodes.workload(workload)
    say("blocked kernel on", workload, ns.n_nodes, "nodes")
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, n)
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=m, n=n)
    w, st, nbr = host(w), host(st), host(NB)
    del X, Y, NB
    assert np.all(st == 0)
    step = max(1, ns.n_nodes // 200)
    rows = np.unique(np.concatenate([np.arange(0, ns.n_nodes, step), [ns.n_nodes - 1]]))
    nbr_ref = oracle.knn(ns.x, ns.y, n, queries=rows)
    assert np.array_equal(nbr[rows], nbr_ref)
    full = np.zeros((ns.n_nodes, n), dtype=np.int32)
    full[rows] = nbr_ref
    w_ref, st_ref = oracle.weights(ns.x, ns.y, full, m=m, n=n, rows=rows)
    assert np.all(st_ref == 0)
    assert np.array_equal(w[rows], w_ref)
    # at every row: the weights annihilate constants
    assert np.all(np.abs(w.sum(axis=1)) <= 1e-9 * np.abs(w).sum(axis=1))
