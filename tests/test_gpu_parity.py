"""GPU vs oracle parity, through the C ABI (Python binding).

Inputs are seeded node sets; the oracle computes its own supports and
weights, and nothing the GPU returns is ever fed to the oracle.  Bars:
kNN, CSR structure and values, SpMV: bit-exact (same definitions, same
operation order).  Weights (FP64): per-stencil relative error
max_k |w_gpu - w_ref| / max_k |w_ref| <= 1e-11; the kernels follow the
reference's operation sequence, so most stencils agree to the last bit and
the test reports that fraction too.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu
TOL_W = 1e-11
NFM = {2: 12, 4: 30, 6: 56}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_err(w_gpu, w_ref, n):
    a, b = w_gpu[:, :n], w_ref[:, :n]
    return np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


# ---------------------------------------------------------------- kNN -----
def _lattice_shuffled():
    g = np.arange(9, dtype=np.float64)
    X, Y = np.meshgrid(g, g)
    perm = np.random.default_rng(3).permutation(81)
    return X.ravel()[perm].copy(), Y.ravel()[perm].copy()


@pytest.mark.parametrize("case,k", [("square45", 12), ("disk3000", 30), ("cc100", 56),
                                    ("lattice", 13), ("dups", 9), ("nan", 8), ("tiny", 5)])
def test_knn_bit_exact(case, k):
    say("knn", case, k)
    if case == "square45":
        ns = nodes.unit_square(45, 1); x, y = ns.x, ns.y
    elif case == "disk3000":
        ns = nodes.unit_disk(3000, 200, seed=21); x, y = ns.x, ns.y
    elif case == "cc100":
        ns = nodes.cell_centred_square(100, seed=4); x, y = ns.x, ns.y
    elif case == "lattice":
        x, y = _lattice_shuffled()
    elif case == "dups":
        ns = nodes.unit_square(10, 2)
        x = np.concatenate([ns.x, ns.x[:7]]); y = np.concatenate([ns.y, ns.y[:7]])
    elif case == "nan":
        ns = nodes.unit_square(8, 4); x, y = ns.x.copy(), ns.y.copy(); x[5] = np.nan
    else:
        x = np.array([0.0, 1.0, 0.5, 0.25, 2.0]); y = np.array([0.0, 0.0, 1.0, 0.5, -1.0])
    ref = oracle.knn(x, y, k)
    got = host(rb.rbffd_knn(dev(x), dev(y), k))
    assert np.array_equal(got, ref)


def test_knn_full_size_disk_sampled_rows():
    ns = nodes.workload("disk_100k_m4")
    say("knn disk 100k", ns.n_nodes)
    got = host(rb.rbffd_knn(dev(ns.x), dev(ns.y), 30))
    rows = np.unique(np.concatenate([np.arange(0, ns.n_nodes, 97), [ns.n_nodes - 1]]))
    ref = oracle.knn(ns.x, ns.y, 30, queries=rows)
    assert np.array_equal(got[rows], ref)
    # properties at every row: self first, ascending keys, all distinct
    assert np.all(got[:, 0] == np.arange(ns.n_nodes))
    d2 = (ns.x[got] - ns.x[:, None]) ** 2 + (ns.y[got] - ns.y[:, None]) ** 2
    assert np.all(np.diff(d2, axis=1) >= 0)
    s = np.sort(got, axis=1)
    assert np.all(np.diff(s, axis=1) > 0)


# ------------------------------------------------------------ weights -----
@pytest.fixture(scope="module")
def disk_small():
    ns = nodes.unit_disk(3000, 200, seed=21)
    return ns, oracle.knn(ns.x, ns.y, 64)


@pytest.mark.parametrize("m,n,ks", [(2, 12, 12), (4, 30, 30), (6, 56, 56), (2, 12, 40),
                                    (2, 6, 6), (2, 20, 20), (4, 40, 44), (6, 36, 36),
                                    (6, 60, 64)])
def test_weights_match_oracle(disk_small, m, n, ks):
    ns, nbr_all = disk_small
    say("weights", m, n, ks)
    nbr = np.ascontiguousarray(nbr_all[:, :ks])
    w_ref, st_ref = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    w, st, _ = rb.rbffd_weights(dev(ns.x), dev(ns.y), dev(nbr), m=m, n=n)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    ok = st_ref == 0
    e = rel_err(w[ok], w_ref[ok], n)
    exact = np.mean(np.all(w[ok][:, :n] == w_ref[ok][:, :n], axis=1))
    say(f"  max rel err {e.max():.3e}, bit-exact stencils {exact:.4f}")
    assert e.max() <= TOL_W
    assert np.all(w[:, n:] == 0.0)


def test_weights_status_codes():
    ns = nodes.unit_square(8, seed=3)
    x, y = ns.x.copy(), ns.y.copy()
    nbr = oracle.knn(x, y, 12)
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]            # duplicate support node
    nb[11, 3] = x.size + 4           # out of range
    nb[12, 0] = -1
    xx = x.copy()
    xx[nbr[13, 2]] = np.inf          # non-finite coordinate
    w_ref, st_ref = oracle.weights(xx, y, nb, m=2, n=12)
    w, st, _ = rb.rbffd_weights(dev(xx), dev(y), dev(nb), m=2, n=12)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    assert set(st_ref[[10, 11, 12, 13]]) == {5, 4, 3}
    assert np.array_equal(np.isnan(w), np.isnan(w_ref))
    good = st_ref == 0
    assert rel_err(w[good], w_ref[good], 12).max() <= TOL_W
    # collinear support: the P block is rank deficient -> zero pivot
    xl = np.linspace(0.0, 1.0, 6)
    yl = np.full(6, 0.25)
    nl = np.tile(np.arange(6, dtype=np.int32), (6, 1))
    _, st_ref = oracle.weights(xl, yl, nl, m=2, n=6)
    w, st, _ = rb.rbffd_weights(dev(xl), dev(yl), dev(nl), m=2, n=6)
    assert np.array_equal(host(st), st_ref)
    assert np.all(st_ref == oracle.SINGULAR)
    assert np.all(np.isnan(host(w)))


@pytest.mark.parametrize("m,n", [(2, 12), (4, 30), (6, 56), (4, 40), (2, 20)])
def test_weights_overflowing_offset(m, n):
    """A support node 1e200 away (its offset's square overflows, the scale
    is +inf): every kernel fails the stencil NONFINITE as the oracle does,
    in FP64, with the factors saved and in mixed precision."""
    ns = nodes.unit_square(14, seed=4)
    x = np.append(ns.x, 1e200)
    y = np.append(ns.y, 0.5)
    nbr = np.ascontiguousarray(oracle.knn(x, y, n))  # the far node's own stencil too
    rows = [5, 17, 40]
    nbr[rows, n - 1] = x.size - 1
    w_ref, st_ref = oracle.weights(x, y, nbr, m=m, n=n)
    assert np.all(st_ref[rows] == oracle.NONFINITE) and st_ref[-1] == oracle.NONFINITE
    variants = [{}]
    if (m, n) in ((2, 12), (4, 30), (6, 56)):
        variants += [{"save": True}, {"precision": rb.MIXED}]
    for kw in variants:
        say("overflowing offset", m, n, kw)
        w, st, _ = rb.rbffd_weights(dev(x), dev(y), dev(nbr), m=m, n=n, **kw)
        w, st = host(w), host(st)
        if "precision" in kw:
            st = np.where(st == rb.FELL_BACK_FP64, 0, st)
        assert np.array_equal(st, st_ref), kw
        assert np.array_equal(np.isnan(w[:, :n]), np.isnan(w_ref[:, :n])), kw


def test_weights_mixed_order_matches_oracle():
    ns = nodes.cell_centred_square(60, seed=3, order_seed=33)
    say("weights mixed order", ns.n_nodes)
    nbr = oracle.knn(ns.x, ns.y, 56)
    w_ref, st_ref = oracle.weights(ns.x, ns.y, nbr, order=ns.order)
    w, st, _ = rb.rbffd_weights(dev(ns.x), dev(ns.y), dev(nbr), order=dev(ns.order))
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    for m in (2, 4, 6):
        sel = ns.order == m
        assert rel_err(w[sel], w_ref[sel], NFM[m]).max() <= TOL_W
        assert np.all(w[sel][:, NFM[m]:] == 0.0)
    bad = ns.order.copy()
    bad[7] = 3
    w, st, _ = rb.rbffd_weights(dev(ns.x), dev(ns.y), dev(nbr), order=dev(bad))
    st = host(st)
    assert st[7] == rb.BAD_ORDER and np.all(np.isnan(host(w)[7]))


def test_weights_full_size_disk_sampled():
    ns = nodes.workload("disk_100k_m4")
    say("weights disk 100k m=4", ns.n_nodes)
    X, Y = dev(ns.x), dev(ns.y)
    nbr_g = rb.rbffd_knn(X, Y, 30)
    w, st, _ = rb.rbffd_weights(X, Y, nbr_g, m=4, n=30)
    w, st, nbr_h = host(w), host(st), host(nbr_g)
    assert np.all(st == 0)
    rows = np.unique(np.concatenate([np.arange(0, ns.n_nodes, 211), [ns.n_nodes - 1]]))
    nbr_ref = oracle.knn(ns.x, ns.y, 30, queries=rows)
    assert np.array_equal(nbr_h[rows], nbr_ref)
    full = np.zeros((ns.n_nodes, 30), dtype=np.int32)
    full[rows] = nbr_ref
    w_ref, st_ref = oracle.weights(ns.x, ns.y, full, m=4, n=30, rows=rows)
    assert np.all(st_ref == 0)
    assert rel_err(w[rows], w_ref, 30).max() <= TOL_W
    # a property at every row: the weights annihilate constants
    assert np.all(np.abs(w.sum(axis=1)) <= 1e-10 * np.abs(w).sum(axis=1))


# ------------------------------------------------------------ CSR/SpMV ----
def test_csr_and_spmv_bit_exact():
    ns = nodes.unit_square(45, 1)
    nbr = oracle.knn(ns.x, ns.y, 12)
    w_ref, _ = oracle.weights(ns.x, ns.y, nbr, m=2, n=12)
    rp_ref, col_ref, val_ref = oracle.csr(nbr, w_ref, n=12, is_boundary=ns.is_boundary)
    rp, col, val = rb.rbffd_assemble_csr(dev(nbr), dev(w_ref), n=12,
                                         is_boundary=dev(ns.is_boundary))
    rp, col, val = host(rp), host(col), host(val)
    nnz = int(rp[-1])
    assert np.array_equal(rp, rp_ref)
    assert np.array_equal(col[:nnz], col_ref)
    assert np.array_equal(val[:nnz], val_ref)
    u, f = nodes.manufactured(ns.x, ns.y)
    y_ref = oracle.spmv(rp_ref, col_ref, val_ref, u, f)
    y = host(rb.rbffd_spmv(dev(rp_ref), dev(col_ref), dev(val_ref), dev(u), dev(f)))
    assert np.array_equal(y, y_ref)
    y0 = host(rb.rbffd_spmv(dev(rp_ref), dev(col_ref), dev(val_ref), dev(u)))
    assert np.array_equal(y0, oracle.spmv(rp_ref, col_ref, val_ref, u))


def test_csr_mixed_order_bit_exact():
    ns = nodes.cell_centred_square(40, seed=3, order_seed=33)
    nbr = oracle.knn(ns.x, ns.y, 56)
    w_ref, _ = oracle.weights(ns.x, ns.y, nbr, order=ns.order)
    bnd = (np.arange(ns.n_nodes) % 17 == 0).astype(np.uint8)
    rp_ref, col_ref, val_ref = oracle.csr(nbr, w_ref, order=ns.order, is_boundary=bnd)
    rp, col, val = rb.rbffd_assemble_csr(dev(nbr), dev(w_ref), order=dev(ns.order),
                                         is_boundary=dev(bnd))
    rp, col, val = host(rp), host(col), host(val)
    nnz = int(rp[-1])
    assert np.array_equal(rp, rp_ref)
    assert np.array_equal(col[:nnz], col_ref)
    assert np.array_equal(val[:nnz], val_ref)


def test_pipeline_square_h45_m2():
    """kNN -> weights -> CSR -> residual W u - f on the GPU, each step against
    the oracle's own pipeline on the same nodes."""
    ns = nodes.workload("square_h45_m2")
    X, Y = dev(ns.x), dev(ns.y)
    nbr = rb.rbffd_knn(X, Y, 12)
    w, st, _ = rb.rbffd_weights(X, Y, nbr, m=2, n=12)
    rp, col, val = rb.rbffd_assemble_csr(nbr, w, n=12, is_boundary=dev(ns.is_boundary))
    u, f = nodes.manufactured(ns.x, ns.y)
    r = rb.rbffd_spmv(rp, col, val, dev(u), dev(f))
    nbr_ref = oracle.knn(ns.x, ns.y, 12)
    w_ref, st_ref = oracle.weights(ns.x, ns.y, nbr_ref, m=2, n=12)
    rp_ref, col_ref, val_ref = oracle.csr(nbr_ref, w_ref, n=12, is_boundary=ns.is_boundary)
    r_ref = oracle.spmv(rp_ref, col_ref, val_ref, u, f)
    assert np.array_equal(host(nbr), nbr_ref)
    assert np.array_equal(host(st), st_ref)
    e = rel_err(host(w), w_ref, 12)
    assert e.max() <= TOL_W
    if np.array_equal(host(w), w_ref):
        assert np.array_equal(host(r), r_ref)
    else:
        scale = np.abs(val_ref).max() * np.abs(u).max() * 12
        assert np.abs(host(r) - r_ref).max() <= 1e-12 * scale
