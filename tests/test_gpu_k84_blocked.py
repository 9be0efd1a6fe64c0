"""K = 84 (m = 6, n = 56) weights from the blocked kernel whose trailing
updates run on the matrix cores, against the oracle and against the
unblocked column-split kernel (the path taken when the factors are saved
for the adjoint).

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


def both_paths(x, y, nbr):
    X, Y, NB = dev(x), dev(y), dev(nbr)
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=6, n=56)             # blocked, MFMA
    w2, st2, _ = rb.rbffd_weights(X, Y, NB, m=6, n=56, save=True)  # column-split
    return host(w), host(st), host(w2), host(st2)


def check_same(x, y, nbr, label):
    w_ref, st_ref = oracle.weights(x, y, nbr, m=6, n=56)
    w, st, w2, st2 = both_paths(x, y, nbr)
    say(label, "stencils", nbr.shape[0], "statuses", np.bincount(st_ref))
    assert np.array_equal(st, st_ref)
    assert np.array_equal(st2, st_ref)
    assert np.array_equal(w, w2, equal_nan=True)
    ok = st_ref == 0
    assert np.array_equal(w[ok], w_ref[ok])
    assert np.all(np.isnan(w[~ok]))
    assert np.all(w[ok][:, 56:] == 0.0)


def test_blocked_k84_disk_bit_exact():
    ns = nodes.unit_disk(3000, 200, seed=21)
    nbr = oracle.knn(ns.x, ns.y, 64)
    check_same(ns.x, ns.y, np.ascontiguousarray(nbr[:, :56]), "disk 3200, k_stride 56")
    # a wider row stride (zeros past n)
    check_same(ns.x, ns.y, nbr, "disk 3200, k_stride 64")


def test_blocked_k84_exact_lattice_ties():
    # an unjittered lattice: many entries of equal magnitude, so the pivot
    # search takes its exact (|a|, position) path often
    ns = nodes.cell_centred_square(24, seed=7, jitter=0.0)
    nbr = oracle.knn(ns.x, ns.y, 56)
    check_same(ns.x, ns.y, nbr, "exact lattice 24x24")


def test_blocked_k84_status_codes():
    ns = nodes.unit_square(12, seed=3)
    x, y = ns.x.copy(), ns.y.copy()
    nbr = oracle.knn(x, y, 56)
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]            # duplicate support node
    nb[11, 30] = x.size + 4          # out of range
    nb[12, 55] = -1
    xx = x.copy()
    xx[nbr[13, 40]] = np.inf         # non-finite coordinate
    check_same(xx, y, nb, "status codes")
    # collinear support: the P block is rank deficient -> zero pivot
    xl = np.linspace(0.0, 1.0, 60)
    yl = np.full(60, 0.25)
    nl = np.tile(np.arange(56, dtype=np.int32), (60, 1))
    w_ref, st_ref = oracle.weights(xl, yl, nl, m=6, n=56)
    assert np.all(st_ref == oracle.SINGULAR)
    w, st, w2, st2 = both_paths(xl, yl, nl)
    assert np.array_equal(st, st_ref) and np.array_equal(st2, st_ref)
    assert np.all(np.isnan(w))


def test_blocked_k84_full_size_sampled():
    # 1M-node square, m = 6, in the launch the benchmark times
    ns = nodes.workload("square_1m_m6")
    say("blocked K=84 on", ns.n_nodes, "nodes")
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, 56)
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=6, n=56)
    w, st, nbr = host(w), host(st), host(NB)
    del X, Y, NB
    assert np.all(st == 0)
    rows = np.unique(np.concatenate([np.arange(0, ns.n_nodes, 4999), [ns.n_nodes - 1]]))
    nbr_ref = oracle.knn(ns.x, ns.y, 56, queries=rows)
    assert np.array_equal(nbr[rows], nbr_ref)
    full = np.zeros((ns.n_nodes, 56), dtype=np.int32)
    full[rows] = nbr_ref
    w_ref, st_ref = oracle.weights(ns.x, ns.y, full, m=6, n=56, rows=rows)
    assert np.all(st_ref == 0)
    assert np.array_equal(w[rows], w_ref)
    # at every row: the weights annihilate constants
    assert np.all(np.abs(w.sum(axis=1)) <= 1e-9 * np.abs(w).sum(axis=1))
