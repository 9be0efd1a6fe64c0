"""First-derivative weights (d/dx, d/dy) of eq. (1) from rbffd_weights_op,
against the oracle's weights for the same operator.

The kernels are the Laplacian's with another right-hand side and scale, so
the bar is the Laplacian's: every weight the same double as the oracle's
(NaN where the stencil failed), every status the same.  At the full
100,000-node size the oracle is run on a sample of rows, and the
polynomial reproduction of eq. (1) (the weights differentiate every
polynomial of degree <= m exactly) is checked on every row.
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu

ORDERS = [(2, 12), (4, 30), (6, 56)]
OPS = [(rb.OP_DX, oracle.D_DX, "d/dx"), (rb.OP_DY, oracle.D_DY, "d/dy")]


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


def check_op(x, y, nbr, m, n, op, oop, label):
    w_ref, st_ref = oracle.weights_op(x, y, nbr, m, n, oop)
    say(label, f"m={m}", "stencils", nbr.shape[0], "statuses", np.bincount(st_ref))
    w, st = rb.rbffd_weights_op(dev(x), dev(y), dev(nbr), m, n, op)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    ok = st_ref == 0
    assert np.array_equal(w[ok], w_ref[ok])
    assert np.all(np.isnan(w[~ok]))
    assert np.all(w[ok][:, n:] == 0.0)
    return w, st


@pytest.mark.parametrize("m,n", ORDERS)
@pytest.mark.parametrize("op,oop,name", OPS)
def test_op_disk_bit_exact(m, n, op, oop, name):
    ns = nodes.unit_disk(3000, 200, seed=31)
    nbr = oracle.knn(ns.x, ns.y, 64)
    check_op(ns.x, ns.y, np.ascontiguousarray(nbr[:, :n]), m, n, op, oop,
             f"{name} disk 3200, k_stride {n}")
    check_op(ns.x, ns.y, nbr, m, n, op, oop, f"{name} disk 3200, k_stride 64")


@pytest.mark.parametrize("m,n", ORDERS)
def test_op_lattice_ties(m, n):
    # an unjittered lattice: many entries of equal magnitude, so the pivot
    # search meets ties that both sides must break alike
    g = np.arange(40, dtype=np.float64) / 39.0
    X, Y = np.meshgrid(g, g)
    x, y = X.ravel().copy(), Y.ravel().copy()
    nbr = np.ascontiguousarray(oracle.knn(x, y, n))
    for op, oop, name in OPS:
        check_op(x, y, nbr, m, n, op, oop, f"{name} lattice 1600")


@pytest.mark.parametrize("m,n", ORDERS)
def test_op_status_codes(m, n):
    ns = nodes.unit_square(12, seed=3)
    x, y = ns.x.copy(), ns.y.copy()
    nbr = oracle.knn(x, y, n)
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]            # duplicate support node
    nb[11, n // 2] = x.size + 4      # out of range
    nb[12, n - 1] = -1
    xx = x.copy()
    xx[nbr[13, n - 3]] = np.inf      # non-finite coordinate
    for op, oop, name in OPS:
        w, st = check_op(xx, y, nb, m, n, op, oop, f"{name} status codes")
        assert np.all(st[10:14] != 0)
    # collinear support: the P block is rank deficient -> zero pivot
    xl = np.linspace(0.0, 1.0, n + 4)
    yl = np.full(n + 4, 0.25)
    nl = np.tile(np.arange(n, dtype=np.int32), (n + 4, 1))
    for op, oop, name in OPS:
        w, st = check_op(xl, yl, nl, m, n, op, oop, f"{name} collinear")
        assert np.all(st == oracle.SINGULAR)


def test_op_laplacian_is_weights():
    ns = nodes.unit_disk(2000, 150, seed=32)
    nbr = np.ascontiguousarray(oracle.knn(ns.x, ns.y, 30))
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    w0, st0 = rb.rbffd_weights_op(X, Y, NB, 4, 30, rb.OP_LAPLACIAN)
    w1, st1, _ = rb.rbffd_weights(X, Y, NB, m=4, n=30)
    assert np.array_equal(host(st0), host(st1))
    assert np.array_equal(host(w0), host(w1), equal_nan=True)


def test_op_argument_errors():
    ns = nodes.unit_disk(500, 60, seed=33)
    nbr = np.ascontiguousarray(oracle.knn(ns.x, ns.y, 40))
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    with pytest.raises(rb.RbffdError, match=r"-3"):      # K = 70 + 28 = 98 > 96
        NB70 = dev(np.zeros((ns.n_nodes, 70), np.int32))
        rb.rbffd_weights_op(X, Y, NB70, 6, 70, rb.OP_DX)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # unknown operator
        rb.rbffd_weights_op(X, Y, NB, 4, 30, 3)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # n above the row stride
        rb.rbffd_weights_op(X, Y, NB[:, :12].contiguous(), 4, 30, rb.OP_DY)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # n below the monomial count
        rb.rbffd_weights_op(X, Y, NB, 6, 20, rb.OP_DY)


@pytest.mark.parametrize("m,n", [(4, 30), (6, 56)])
def test_op_full_size_sampled(m, n):
    # the 100,000-node disk the timed path runs on, one launch of every row
    ns = nodes.unit_disk(100_000, 2_000, seed=7)
    X, Y = dev(ns.x), dev(ns.y)
    nb_t = rb.rbffd_knn(X, Y, n)
    nbr = host(nb_t)
    rng = np.random.default_rng(34)
    rows = np.sort(rng.choice(ns.x.shape[0], 300, replace=False))
    for op, oop, name in OPS:
        w_t, st_t = rb.rbffd_weights_op(X, Y, nb_t, m, n, op)
        w, st = host(w_t), host(st_t)
        w_ref, st_ref = oracle.weights_op(ns.x, ns.y, nbr, m, n, oop, rows=rows)
        say(name, f"m={m}", "full 102000, sampled", rows.size, "failed", int((st != 0).sum()))
        assert np.array_equal(st[rows], st_ref)
        assert np.array_equal(w[rows], w_ref, equal_nan=True)
        assert np.all(st == 0)
        # every row: exact on the polynomial dx^a dy^b (a + b <= m) about the
        # centre, to a residual small beside the terms it sums.
        dx = ns.x[nbr] - ns.x[:, None]
        dy = ns.y[nbr] - ns.y[:, None]
        for a in range(m + 1):
            for b in range(m + 1 - a):
                f = dx ** a * dy ** b
                got = (w * f).sum(axis=1)
                want = 1.0 if (op == rb.OP_DX and (a, b) == (1, 0)) or \
                    (op == rb.OP_DY and (a, b) == (0, 1)) else 0.0
                rel = np.abs(got - want) / (np.abs(w * f).sum(axis=1) + want)
                assert rel.max() < 1e-9, (name, a, b, rel.max())


# supports other than the standard three: the padded instances (K <= 32,
# K <= 64: the multi-slot kernel; K <= 96: the two-wavefront kernel)
PADDED = [(2, 6), (2, 20), (4, 20), (4, 40), (6, 36), (6, 60), (4, 64)]


@pytest.mark.parametrize("m,n", PADDED)
def test_op_padded_supports(m, n):
    ns = nodes.unit_disk(3000, 200, seed=34)
    nbr = oracle.knn(ns.x, ns.y, 72)
    for ks in (n, 72):
        nb = np.ascontiguousarray(nbr[:, :ks])
        for op, oop, name in OPS:
            w_ref, st_ref = oracle.weights_op(ns.x, ns.y, nb, m, n, oop)
            w, st = rb.rbffd_weights_op(dev(ns.x), dev(ns.y), dev(nb), m, n, op)
            w, st = host(w), host(st)
            ok = st_ref == 0
            a, b = w[ok][:, :n], w_ref[ok][:, :n]
            rel = np.abs(a - b).max(axis=1) / np.abs(b).max(axis=1)
            exact = np.mean(np.all(a == b, axis=1))
            say(f"{name} m={m} n={n} k_stride={ks}: statuses {np.bincount(st_ref)}, "
                f"max rel err {rel.max():.2e}, bit-exact stencils {exact:.4f}")
            assert np.array_equal(st, st_ref)
            assert rel.max() <= 1e-11
            assert np.all(np.isnan(w[~ok][:, :n]))
            assert np.all(w[:, n:] == 0.0)


# ---- mixed-order batch of the derivative operators (rbffd_weights_op_batch)

def _op_batch_ref(x, y, nbr, order, oop):
    """The oracle's weights at each node's order on the standard supports;
    NaN weights and BAD_ORDER where the order is not 2, 4 or 6."""
    N, ks = nbr.shape
    w = np.full((N, ks), np.nan)
    st = np.full(N, rb.BAD_ORDER, np.int32)
    for m, n in ((2, 12), (4, 30), (6, 56)):
        rows = np.nonzero(order == m)[0]
        if rows.size:
            w[rows], st[rows] = oracle.weights_op(x, y, nbr, m, n, oop, rows=rows)
    return w, st


@pytest.mark.parametrize("op,oop,name", OPS)
@pytest.mark.parametrize("mix", ["mixed", "bad"])
def test_op_batch_bit_exact(op, oop, name, mix):
    """Per-node orders on a 3200-node disk with a stride of 60 columns:
    every node's weights and status are the oracle's at its order."""
    ns = nodes.unit_disk(3000, 200, seed=36)
    nbr = oracle.knn(ns.x, ns.y, 60)
    rng = np.random.default_rng(37)
    vals = [2, 4, 6] if mix == "mixed" else [2, 4, 6, 3, 0, 8]
    order = rng.choice(np.array(vals, np.int8), ns.n_nodes)
    say(name, "batch", mix, ns.n_nodes)
    w_ref, st_ref = _op_batch_ref(ns.x, ns.y, nbr, order, oop)
    w, st = rb.rbffd_weights_op_batch(dev(ns.x), dev(ns.y), dev(nbr), dev(order), op)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    assert np.array_equal(w, w_ref, equal_nan=True)


def test_op_batch_full_size_matches_single_order():
    """The 1M-node square with orders uniform on {2, 4, 6}: the batch's d/dx
    weights are the single-order launches' at each node's order, bit for
    bit, on every row."""
    ns = nodes.workload("square_1m_mixed")
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, 56)
    say("d/dx batch square", ns.n_nodes)
    w_b, st_b = rb.rbffd_weights_op_batch(X, Y, NB, dev(ns.order), rb.OP_DX)
    assert int((st_b != 0).sum().item()) == 0
    for m, n in ((2, 12), (4, 30), (6, 56)):
        sel = torch.as_tensor(ns.order == m).cuda()
        w_s, _ = rb.rbffd_weights_op(X, Y, NB[:, :n].contiguous(), m, n, rb.OP_DX)
        assert torch.equal(w_b[sel][:, :n], w_s[sel]), m
        assert torch.all(w_b[sel][:, n:] == 0.0)
        del w_s


def test_op_batch_argument_errors():
    ns = nodes.unit_disk(300, 40, seed=38)
    nbr = oracle.knn(ns.x, ns.y, 56)
    X, Y = dev(ns.x), dev(ns.y)
    order = dev(np.full(ns.n_nodes, 4, np.int8))
    with pytest.raises(ValueError):  # fewer than 56 columns
        rb.rbffd_weights_op_batch(X, Y, dev(nbr[:, :40]), order, rb.OP_DX)
    with pytest.raises(rb.RbffdError):  # the Laplacian batch is rbffd_weights
        rb.rbffd_weights_op_batch(X, Y, dev(nbr), order, rb.OP_LAPLACIAN)
    lib = rb._load()
    NB = dev(nbr)
    w = torch.empty((ns.n_nodes, 56), dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    rc = lib.rbffd_weights_op_batch(rb._p(X), rb._p(Y), ns.n_nodes, rb._p(NB), 56, rb._p(order),
                                    rb.OP_DX, rb._p(w), None, rb._p(ws), 16, rb._stream(X.device))
    assert rc == -2  # RBFFD_ERR_WORKSPACE
