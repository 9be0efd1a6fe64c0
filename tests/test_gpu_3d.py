"""Three-dimensional supports (rbffd_knn3), Laplacian weights
(rbffd_weights3) and first-derivative weights (rbffd_weights3_op) against the
oracle's knn3 / weights3 / weights3_op.

kNN is compared index for index.  The weights take the same operations in
the same order as the oracle's LU and solves, so they are compared double
for double (NaN where the stencil failed), status for status.  At the full
size (a jittered 100^3 lattice, one launch of every row) the oracle runs on
sampled rows, and every row is checked for exact reproduction of the
quadratics (the polynomial part of eq. (1)).
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


def lattice_with_ties():
    g = np.arange(7, dtype=np.float64)
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    x[5], y[5], z[5] = x[9], y[9], z[9]   # a duplicate node
    z[11] = np.nan                        # never selected
    return x, y, z


@pytest.mark.parametrize("k", [1, 10, 20, 27, 33, 45, 64, 65, 70, 80, 100, 128])
def test_knn3_bit_exact(k):
    x, y, z = nodes.jittered_cube(12, seed=21)
    say("knn3 cube 1728", k)
    ref = oracle.knn3(x, y, z, k)
    got = host(rb.rbffd_knn3(dev(x), dev(y), dev(z), k))
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("k", [7, 20, 33, 70, 128])
def test_knn3_ties_dups_nan(k):
    x, y, z = lattice_with_ties()
    say("knn3 lattice 343 with ties", k)
    ref = oracle.knn3(x, y, z, k)
    got = host(rb.rbffd_knn3(dev(x), dev(y), dev(z), k))
    assert np.array_equal(got, ref)


def test_knn3_flat_and_tiny():
    # coplanar nodes (a flat bounding box) and a set of exactly k nodes
    rng = np.random.default_rng(5)
    x, y = rng.random(500), rng.random(500)
    z = np.zeros(500)
    say("knn3 flat 500")
    assert np.array_equal(host(rb.rbffd_knn3(dev(x), dev(y), dev(z), 20)),
                          oracle.knn3(x, y, z, 20))
    x, y, z = rng.random((3, 6))
    assert np.array_equal(host(rb.rbffd_knn3(dev(x), dev(y), dev(z), 6)),
                          oracle.knn3(x, y, z, 6))
    # exactly k nodes with the one-wavefront-per-query kernel (k > 32)
    x, y, z = rng.random((3, 90))
    assert np.array_equal(host(rb.rbffd_knn3(dev(x), dev(y), dev(z), 90)),
                          oracle.knn3(x, y, z, 90))


def check_weights3(x, y, z, nbr, n, label, m=2):
    w_ref, st_ref = oracle.weights3(x, y, z, nbr, m, n)
    say(label, "m", m, "n", n, "stencils", nbr.shape[0], "statuses", np.bincount(st_ref))
    w, st = rb.rbffd_weights3(dev(x), dev(y), dev(z), dev(nbr), m, n)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    ok = st_ref == 0
    assert np.array_equal(w[ok], w_ref[ok])
    assert np.all(np.isnan(w[~ok][:, :n]))
    assert np.all(w[:, n:] == 0.0)
    return w, st


@pytest.mark.parametrize("n", [10, 20, 22, 23, 40, 54])
def test_weights3_bit_exact(n):
    x, y, z = nodes.jittered_cube(11, seed=22)
    nbr = oracle.knn3(x, y, z, 64)
    check_weights3(x, y, z, np.ascontiguousarray(nbr[:, :n]), n, "cube 1331, k_stride n")
    check_weights3(x, y, z, nbr, n, "cube 1331, k_stride 64")


@pytest.mark.parametrize("n", [20, 40])
def test_weights3_lattice_ties(n):
    g = np.arange(9, dtype=np.float64) / 8.0
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    nbr = np.ascontiguousarray(oracle.knn3(x, y, z, n))
    check_weights3(x, y, z, nbr, n, "exact lattice 729")


@pytest.mark.parametrize("n", [20, 40])
def test_weights3_status_codes(n):
    x, y, z = nodes.jittered_cube(6, seed=23)
    nbr = oracle.knn3(x, y, z, n)
    nb = nbr.copy()
    nb[3, 4] = nb[3, 2]             # duplicate support node
    nb[4, 7] = len(x) + 1           # out of range
    nb[5, n - 1] = -1
    xx = x.copy()
    xx[nbr[6, 5]] = np.inf          # non-finite coordinate
    w, st = check_weights3(xx, y, z, nb, n, "status codes")
    assert np.all(st[3:7] != 0)
    # coplanar supports: the z monomials vanish -> zero pivot
    rng = np.random.default_rng(6)
    xp, yp = rng.random(200), rng.random(200)
    zp = np.full(200, 0.5)
    nbp = np.ascontiguousarray(oracle.knn3(xp, yp, zp, n))
    w, st = check_weights3(xp, yp, zp, nbp, n, "coplanar")
    assert np.all(st == oracle.SINGULAR)


def test_weights3_argument_errors():
    x, y, z = nodes.jittered_cube(5, seed=24)
    nbr = np.ascontiguousarray(oracle.knn3(x, y, z, 64))
    X, Y, Z, NB = dev(x), dev(y), dev(z), dev(nbr)
    with pytest.raises(rb.RbffdError, match=r"-3"):      # K = 70 > 64
        rb.rbffd_weights3(X, Y, Z, NB, 2, 60)
    with pytest.raises(rb.RbffdError, match=r"-3"):      # m = 4: n <= 76 (K <= 111)
        NB80 = dev(np.zeros((x.size, 80), np.int32))
        rb.rbffd_weights3(X, Y, Z, NB80, 4, 77)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # m = 2 or 4
        rb.rbffd_weights3(X, Y, Z, NB, 3, 40)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # m = 4: n below 35 monomials
        rb.rbffd_weights3(X, Y, Z, NB, 4, 30)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # n below the monomial count
        rb.rbffd_weights3(X, Y, Z, NB, 2, 9)
    with pytest.raises(rb.RbffdError, match=r"-1"):      # n above the row stride
        rb.rbffd_weights3(X, Y, Z, NB[:, :12].contiguous(), 2, 20)


def test_3d_full_size_sampled():
    x, y, z = nodes.jittered_cube(100, seed=6)
    N = x.shape[0]
    say("3-D cube", N, "k = n = 20")
    X, Y, Z = dev(x), dev(y), dev(z)
    nb_t = rb.rbffd_knn3(X, Y, Z, 20)
    nbr = host(nb_t)
    rng = np.random.default_rng(25)
    rows = np.sort(rng.choice(N, 200, replace=False))
    assert np.array_equal(nbr[rows], oracle.knn3(x, y, z, 20, queries=rows))
    w_t, st_t = rb.rbffd_weights3(X, Y, Z, nb_t, 2, 20)
    w, st = host(w_t), host(st_t)
    assert np.all(st == 0)
    w_ref, st_ref = oracle.weights3(x, y, z, nbr, 2, 20, rows=rows)
    assert np.array_equal(st[rows], st_ref)
    assert np.array_equal(w[rows], w_ref)
    # every row: the quadratics about the centre, exactly up to rounding
    dx = (x[nbr] - x[:, None]).astype(np.float64)
    dy = y[nbr] - y[:, None]
    dz = z[nbr] - z[:, None]
    for (a, b, c) in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0),
                      (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]:
        f = dx ** a * dy ** b * dz ** c
        want = 2.0 if sorted((a, b, c)) == [0, 0, 2] else 0.0
        got = (w * f).sum(1)
        rel = np.abs(got - want) / ((np.abs(w * f)).sum(1) + want)
        assert rel.max() < 1e-9, ((a, b, c), rel.max())


D3 = [(rb.OP_DX, oracle.D3_DX, (1, 0, 0)), (rb.OP_DY, oracle.D3_DY, (0, 1, 0)),
      (rb.OP3_DZ, oracle.D3_DZ, (0, 0, 1))]


@pytest.mark.parametrize("op,oop,axis", D3)
@pytest.mark.parametrize("n", [20, 40])
def test_weights3_derivatives_bit_exact(op, oop, axis, n):
    x, y, z = nodes.jittered_cube(11, seed=26)
    nbr = oracle.knn3(x, y, z, 64)
    for nb, label in ((np.ascontiguousarray(nbr[:, :n]), "k_stride n"), (nbr, "k_stride 64")):
        w_ref, st_ref = oracle.weights3_op(x, y, z, nb, 2, n, oop)
        say("3-D derivative", axis, "n", n, label)
        w, st = rb.rbffd_weights3(dev(x), dev(y), dev(z), dev(nb), 2, n, op=op)
        w, st = host(w), host(st)
        assert np.array_equal(st, st_ref)
        assert np.array_equal(w, w_ref, equal_nan=True)


def test_weights3_derivatives_full_size_sampled():
    x, y, z = nodes.jittered_cube(100, seed=6)
    N = x.shape[0]
    X, Y, Z = dev(x), dev(y), dev(z)
    nb_t = rb.rbffd_knn3(X, Y, Z, 20)
    nbr = host(nb_t)
    rows = np.sort(np.random.default_rng(27).choice(N, 150, replace=False))
    dx = x[nbr] - x[:, None]
    dy = y[nbr] - y[:, None]
    dz = z[nbr] - z[:, None]
    for op, oop, axis in D3:
        say("3-D derivative full size", axis)
        w_t, st_t = rb.rbffd_weights3(X, Y, Z, nb_t, 2, 20, op=op)
        w, st = host(w_t), host(st_t)
        assert np.all(st == 0)
        w_ref, _ = oracle.weights3_op(x, y, z, nbr, 2, 20, oop, rows=rows)
        assert np.array_equal(w[rows], w_ref)
        for e in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1),
                  (0, 2, 0), (0, 1, 1), (0, 0, 2)]:
            f = dx ** e[0] * dy ** e[1] * dz ** e[2]
            want = 1.0 if e == axis else 0.0
            rel = np.abs((w * f).sum(1) - want) / (np.abs(w * f).sum(1) + want)
            assert rel.max() < 1e-9, (axis, e, rel.max())


def test_weights3_op_argument_errors():
    x, y, z = nodes.jittered_cube(5, seed=24)
    nbr = np.ascontiguousarray(oracle.knn3(x, y, z, 20))
    with pytest.raises(rb.RbffdError, match=r"-1"):
        rb.rbffd_weights3(dev(x), dev(y), dev(z), dev(nbr), 2, 20, op=4)


# ---- m = 4 (K = 105, the blocked LU on the matrix cores) ------------------

MONOS4 = [(a, b, d - a - b) for d in range(5) for a in range(d, -1, -1)
          for b in range(d - a, -1, -1)]


@pytest.mark.parametrize("n", [35, 40, 56, 69, 71, 76])
def test_weights3_m4_other_supports_bit_exact(n):
    """m = 4 on supports other than 70: identity padding to K = 111 in the
    blocked kernel, the oracle's doubles and statuses."""
    x, y, z = nodes.jittered_cube(11, seed=29)
    nbr = oracle.knn3(x, y, z, 80)
    check_weights3(x, y, z, np.ascontiguousarray(nbr[:, :n]), n, f"cube 1331, n {n}", m=4)
    check_weights3(x, y, z, nbr, n, f"cube 1331, n {n}, k_stride 80", m=4)
    for op, oop, axis in D3:
        w_ref, st_ref = oracle.weights3_op(x, y, z, nbr, 4, n, oop)
        w, st = rb.rbffd_weights3(dev(x), dev(y), dev(z), dev(nbr), 4, n, op=op)
        w, st = host(w), host(st)
        assert np.array_equal(st, st_ref)
        assert np.array_equal(w, w_ref, equal_nan=True)


@pytest.mark.parametrize("ks", [70, 80])
def test_weights3_m4_bit_exact(ks):
    x, y, z = nodes.jittered_cube(11, seed=22)
    nbr = oracle.knn3(x, y, z, 80)
    check_weights3(x, y, z, np.ascontiguousarray(nbr[:, :ks]), 70,
                   f"cube 1331, k_stride {ks}", m=4)


def test_weights3_m4_lattice_ties():
    g = np.arange(9, dtype=np.float64) / 8.0
    Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
    x, y, z = X.ravel().copy(), Y.ravel().copy(), Z.ravel().copy()
    nbr = np.ascontiguousarray(oracle.knn3(x, y, z, 70))
    check_weights3(x, y, z, nbr, 70, "exact lattice 729", m=4)


def test_weights3_m4_status_codes():
    x, y, z = nodes.jittered_cube(7, seed=23)
    x, y, z = np.append(x, 1e200), np.append(y, 0.5), np.append(z, 0.5)
    nbr = oracle.knn3(x, y, z, 70)
    nb = nbr.copy()
    nb[3, 4] = nb[3, 2]             # duplicate support node
    nb[4, 7] = len(x) + 1           # out of range
    nb[5, 69] = -1
    nb[7, 69] = len(x) - 1          # a node 1e200 away: the scale overflows
    xx = x.copy()
    xx[nbr[6, 5]] = np.inf          # non-finite coordinate
    w, st = check_weights3(xx, y, z, nb, 70, "status codes", m=4)
    assert np.all(st[3:8] != 0) and st[7] == oracle.NONFINITE and st[-1] == oracle.NONFINITE
    # coplanar supports: the z monomials vanish -> zero pivot
    rng = np.random.default_rng(6)
    xp, yp = rng.random(300), rng.random(300)
    zp = np.full(300, 0.5)
    nbp = np.ascontiguousarray(oracle.knn3(xp, yp, zp, 70))
    w, st = check_weights3(xp, yp, zp, nbp, 70, "coplanar", m=4)
    assert np.all(st == oracle.SINGULAR)


@pytest.mark.parametrize("op,oop,axis", D3)
def test_weights3_m4_derivatives_bit_exact(op, oop, axis):
    x, y, z = nodes.jittered_cube(10, seed=26)
    nbr = oracle.knn3(x, y, z, 72)
    w_ref, st_ref = oracle.weights3_op(x, y, z, nbr, 4, 70, oop)
    say("3-D derivative m = 4", axis)
    w, st = rb.rbffd_weights3(dev(x), dev(y), dev(z), dev(nbr), 4, 70, op=op)
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    assert np.array_equal(w, w_ref, equal_nan=True)


def test_3d_m4_full_size_sampled():
    """The jittered 100^3 lattice, k = n = 70: kNN and weights of sampled
    rows against the oracle, and every row's weights applied to the 35
    monomials of degree <= 4 about its centre (on the device)."""
    x, y, z = nodes.jittered_cube(100, seed=6)
    N = x.shape[0]
    say("3-D cube", N, "m = 4, k = n = 70")
    X, Y, Z = dev(x), dev(y), dev(z)
    nb_t = rb.rbffd_knn3(X, Y, Z, 70)
    rows = np.sort(np.random.default_rng(28).choice(N, 120, replace=False))
    nbr_rows = host(nb_t[torch.as_tensor(rows).cuda()])
    assert np.array_equal(nbr_rows, oracle.knn3(x, y, z, 70, queries=rows))
    w_t, st_t = rb.rbffd_weights3(X, Y, Z, nb_t, 4, 70)
    st = host(st_t)
    assert np.all(st == 0)
    # the oracle on the sampled rows (their supports: the rows above)
    nbr_s = np.zeros((N, 70), np.int32)
    nbr_s[rows] = nbr_rows
    w_ref, st_ref = oracle.weights3(x, y, z, nbr_s, 4, 70, rows=rows)
    assert np.all(st_ref == 0)
    assert np.array_equal(host(w_t[torch.as_tensor(rows).cuda()]), w_ref)
    nbl = nb_t.long()
    dx, dy, dz = X[nbl] - X[:, None], Y[nbl] - Y[:, None], Z[nbl] - Z[:, None]
    worst = 0.0
    for (a, b, c) in MONOS4:
        f = dx ** a * dy ** b * dz ** c
        want = 2.0 if sorted((a, b, c)) == [0, 0, 2] else 0.0
        wf = w_t * f
        rel = (wf.sum(1) - want).abs() / (wf.abs().sum(1) + want)
        worst = max(worst, rel.max().item())
    say("  worst relative residual over the 35 monomials", worst)
    assert worst < 1e-9


# ---- mixed-order batch in three dimensions (rbffd_weights3_batch) --------

def _batch3_ref(x, y, z, nbr, order):
    """The oracle's weights at each node's order (n = 20 for m = 2, 70 for
    m = 4); NaN weights and BAD_ORDER where the order is neither."""
    N, ks = nbr.shape
    w = np.full((N, ks), np.nan)
    st = np.full(N, rb.BAD_ORDER, np.int32)
    for m, n in ((2, 20), (4, 70)):
        rows = np.nonzero(order == m)[0]
        if rows.size:
            w[rows], st[rows] = oracle.weights3(x, y, z, nbr, m, n, rows=rows)
    return w, st


@pytest.mark.parametrize("mix", ["mixed", "all2", "all4", "bad"])
def test_weights3_batch_bit_exact(mix):
    """Per-node orders 2 / 4 (and invalid ones) on a 12^3 jittered lattice
    with a stride of 72 columns: every node's weights and status are the
    oracle's at its order, double for double."""
    x, y, z = nodes.jittered_cube(12, seed=31)
    N = x.shape[0]
    nbr = np.concatenate([oracle.knn3(x, y, z, 70), np.zeros((N, 2), np.int32)], axis=1)
    rng = np.random.default_rng(32)
    order = {"mixed": rng.choice(np.array([2, 4], np.int8), N),
             "all2": np.full(N, 2, np.int8), "all4": np.full(N, 4, np.int8),
             "bad": rng.choice(np.array([2, 4, 3, 0, 6, -1], np.int8), N)}[mix]
    say("3-D batch", mix, N)
    w_ref, st_ref = _batch3_ref(x, y, z, nbr, order)
    w, st = rb.rbffd_weights3_batch(dev(x), dev(y), dev(z), dev(nbr), dev(order))
    w, st = host(w), host(st)
    assert np.array_equal(st, st_ref)
    assert np.array_equal(w, w_ref, equal_nan=True)


def test_weights3_batch_full_size_matches_single_order():
    """The jittered 100^3 lattice with orders drawn uniformly from {2, 4}:
    the batch gives, bit for bit, the single-order launches' weights at each
    node's order, and sampled rows match the oracle."""
    x, y, z = nodes.jittered_cube(100, seed=6)
    N = x.shape[0]
    say("3-D batch cube", N)
    X, Y, Z = dev(x), dev(y), dev(z)
    nb_t = rb.rbffd_knn3(X, Y, Z, 70)
    order = np.random.default_rng(33).choice(np.array([2, 4], np.int8), N)
    O = dev(order)
    w_b, st_b = rb.rbffd_weights3_batch(X, Y, Z, nb_t, O)
    st_b = host(st_b)
    assert np.all(st_b == 0)
    for m, n in ((2, 20), (4, 70)):
        sel = torch.as_tensor(order == m).cuda()
        w_s, st_s = rb.rbffd_weights3(X, Y, Z, nb_t, m, n)
        assert torch.equal(w_b[sel], w_s[sel]), m
        del w_s, st_s
    rows = np.sort(np.random.default_rng(34).choice(N, 60, replace=False))
    nbr_rows = host(nb_t[torch.as_tensor(rows).cuda()])
    nbr_s = np.zeros((N, 70), np.int32)
    nbr_s[rows] = nbr_rows
    w_ref = np.zeros((rows.size, 70))
    for m, n in ((2, 20), (4, 70)):
        pick = order[rows] == m
        if pick.any():
            w_ref[pick], st_r = oracle.weights3(x, y, z, nbr_s, m, n, rows=rows[pick])
            assert np.all(st_r == 0)
    assert np.array_equal(host(w_b[torch.as_tensor(rows).cuda()]), w_ref)


def test_weights3_batch_argument_errors():
    x, y, z = nodes.jittered_cube(5, seed=35)
    N = x.shape[0]
    nbr = oracle.knn3(x, y, z, 70)
    X, Y, Z = dev(x), dev(y), dev(z)
    order = dev(np.full(N, 2, np.int8))
    with pytest.raises(ValueError):  # fewer than 70 columns
        rb.rbffd_weights3_batch(X, Y, Z, dev(nbr[:, :60]), order)
    with pytest.raises(ValueError):  # order of the wrong length
        rb.rbffd_weights3_batch(X, Y, Z, dev(nbr), dev(np.full(N - 1, 2, np.int8)))
    lib = rb._load()
    NB = dev(nbr)
    w = torch.empty((N, 70), dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    rc = lib.rbffd_weights3_batch(rb._p(X), rb._p(Y), rb._p(Z), N, rb._p(NB), 70,
                                  rb._p(order), rb._p(w), None, rb._p(ws), 16,
                                  rb._stream(X.device))
    assert rc == -2  # RBFFD_ERR_WORKSPACE
    rc = lib.rbffd_weights3_batch(rb._p(X), rb._p(Y), rb._p(Z), N, rb._p(NB), 60,
                                  rb._p(order), rb._p(w), None, rb._p(ws), 16,
                                  rb._stream(X.device))
    assert rc == -1  # RBFFD_ERR_ARG
