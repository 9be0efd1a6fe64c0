"""GPU mixed-precision weights (FP32 factorisation + FP64 refinement,
FP64 fallback) against the oracle's mixed form and the FP64 oracle.

m = 2 (K = 18): the GPU performs the same operations in the same precisions
as the oracle's mixed form (FP32 LU and triangular solves with fused
updates, FP64 fused residuals), so weights, statuses (including fall-backs)
and correction counts are compared exactly.

m = 4, 6 (K = 45, 84): the GPU inverts the FP32 system by blocked
Gauss-Jordan on the matrix cores and applies the inverse to each residual;
it is compared with the oracle's Gauss-Jordan form (oracle.MIXED_GJ), whose
FP32 inverse it reproduces bit for bit (the rank-4 matrix-core updates round
as the sequential fused eliminations).  The products with the inverse and
the FP64 residuals sum in another order on the GPU, so a correction's size
can differ in its last bits: statuses must agree, the correction counts of
converged stencils agree for most stencils (all at m = 4, about 85% at
m = 6) and never differ by more than one, and the weights agree to 1e-11
relative (1e-9 against the FP64 oracle, the target).
"""

import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu
NFM = {2: 12, 4: 30, 6: 56}
# the oracle's mixed form that each system size's GPU kernel follows
FORM = {2: oracle.MIXED_LU, 4: oracle.MIXED_GJ, 6: oracle.MIXED_GJ}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel_err(a, b, n):
    return np.abs(a[:, :n] - b[:, :n]).max(axis=1) / np.abs(b[:, :n]).max(axis=1)


def check_mixed(w, st, it, w_mx, st_mx, it_mx, w64, n, exact, what=""):
    """Mixed results against the mixed oracle (exactly when the GPU follows
    the same operations, else to the refinement's accuracy) and the FP64
    oracle (1e-9)."""
    assert np.array_equal(st, st_mx), f"{what}: statuses differ"
    ok = ~np.isnan(w_mx[:, :n]).any(axis=1)
    if exact:
        assert np.array_equal(it, it_mx), f"{what}: correction counts differ"
        assert rel_err(w[ok], w_mx[ok], n).max() <= 1e-12
    else:
        # converged stencils: the same number of corrections, or one more or
        # one fewer where the last correction's size lies at the stopping
        # threshold (the products' summation order moves it by a few ulps);
        # a stencil that falls back reports the corrections it tried before
        # diverging, which such differences can move further
        conv = st_mx == 0
        d = np.abs(it.astype(np.int64) - it_mx)[conv]
        if d.size:
            say(f"  {what}: corrections equal {np.mean(d == 0):.4f}, max diff {d.max()}")
            assert d.max() <= 1 and np.mean(d == 0) >= 0.75, f"{what}: correction counts"
        e_mx = rel_err(w[ok], w_mx[ok], n)
        say(f"  {what}: vs mixed oracle {e_mx.max():.3e}")
        assert e_mx.max() <= 1e-11
    assert np.array_equal(np.isnan(w[:, :n]), np.isnan(w_mx[:, :n]))
    ok64 = ~np.isnan(w64[:, :n]).any(axis=1)
    e64 = rel_err(w[ok64], w64[ok64], n)
    say(f"  {what}: vs FP64 oracle {e64.max():.3e}")
    assert e64.max() <= 1e-9


def gpu_mixed(x, y, nbr, **kw):
    N = nbr.shape[0]
    it = torch.zeros(N, dtype=torch.int32, device="cuda")
    w, st, _ = rb.rbffd_weights(dev(x), dev(y), dev(nbr), precision=rb.MIXED, refine_steps=it, **kw)
    return host(w), host(st), host(it)


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_matches_mixed_oracle_and_fp64(m):
    ns = nodes.unit_disk(3000, 200, seed=21)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n, form=FORM[m])
    w64, st64 = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    w, st, it = gpu_mixed(ns.x, ns.y, nbr, m=m, n=n)
    say("mixed", m, "statuses", np.bincount(st), "mean corrections", it[st == 0].mean(),
        "oracle", it_mx[st_mx == 0].mean())
    check_mixed(w, st, it, w_mx, st_mx, it_mx, w64, n, exact=m == 2, what=f"m={m}")


def test_mixed_fallback_and_failures():
    ns = nodes.unit_square(8, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 12)
    x, y = ns.x.copy(), ns.y.copy()
    i = 30
    x[nbr[i, 4]] = x[nbr[i, 3]] + 1e-4   # ill-conditioned: falls back
    y[nbr[i, 4]] = y[nbr[i, 3]]
    nb = nbr.copy()
    nb[10, 5] = nb[10, 4]                  # duplicate: fails, no fallback
    nb[11, 2] = 10 ** 6                    # bad index
    w_mx, st_mx, it_mx = oracle.weights_mixed(x, y, nb, m=2, n=12)
    w, st, it = gpu_mixed(x, y, nb, m=2, n=12)
    assert st_mx[i] == oracle.FELL_BACK and st_mx[10] == oracle.DUPLICATE
    assert np.array_equal(st, st_mx)
    assert np.array_equal(it, it_mx)
    assert np.array_equal(np.isnan(w), np.isnan(w_mx))
    ok = ~np.isnan(w_mx).any(axis=1)
    assert rel_err(w[ok], w_mx[ok], 12).max() <= 1e-12


def test_mixed_full_size_square_sampled():
    ns = nodes.workload("square_10k_m6")
    say("mixed 10k m=6", ns.n_nodes)
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, 56)
    it = torch.zeros(ns.n_nodes, dtype=torch.int32, device="cuda")
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=6, n=56, precision=rb.MIXED, refine_steps=it)
    w, st, it, nbr = host(w), host(st), host(it), host(NB)
    rows = np.arange(0, ns.n_nodes, 37)
    assert np.array_equal(nbr[rows], oracle.knn(ns.x, ns.y, 56, queries=rows))
    full = np.zeros_like(nbr)
    full[rows] = nbr[rows]
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, full, m=6, n=56, rows=rows,
                                              form=oracle.MIXED_GJ)
    w64, _ = oracle.weights(ns.x, ns.y, full, m=6, n=56, rows=rows)
    check_mixed(w[rows], st[rows], it[rows], w_mx, st_mx, it_mx, w64, 56, exact=False,
                what="10k m=6")
    say("  statuses", np.bincount(st), "mean corrections", it[st == 0].mean())


def test_mixed_order_batch():
    ns = nodes.cell_centred_square(40, seed=3, order_seed=33)
    nbr = oracle.knn(ns.x, ns.y, 56)
    w, st, it = gpu_mixed(ns.x, ns.y, nbr, order=dev(ns.order))
    # per order, the oracle's form that the GPU kernel of that system size runs
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, nbr, order=ns.order)
    w_gj, st_gj, it_gj = oracle.weights_mixed(ns.x, ns.y, nbr, order=ns.order,
                                              form=oracle.MIXED_GJ)
    gj = ns.order != 2
    w_mx[gj], st_mx[gj], it_mx[gj] = w_gj[gj], st_gj[gj], it_gj[gj]
    w64, _ = oracle.weights(ns.x, ns.y, nbr, order=ns.order)
    for m in (2, 4, 6):
        sel = ns.order == m
        check_mixed(w[sel], st[sel], it[sel], w_mx[sel], st_mx[sel], it_mx[sel], w64[sel],
                    NFM[m], exact=m == 2, what=f"batch m={m}")


@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_1m_square_sampled(m):
    """The 1M-node square (h = 1e-3) in mixed precision at m = 2, 4, 6: the
    launches run several grid-stride passes at this size.  Sampled rows
    against the mixed oracle (statuses and corrections exactly) and the FP64
    oracle (1e-9)."""
    ns = nodes.workload("square_1m_m6")
    n = NFM[m]
    say("mixed 1M square m =", m, ns.n_nodes)
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, n)
    it = torch.zeros(ns.n_nodes, dtype=torch.int32, device="cuda")
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=m, n=n, precision=rb.MIXED, refine_steps=it)
    w, st, it, nbr = host(w), host(st), host(it), host(NB)
    assert np.all((st == 0) | (st == rb.FELL_BACK_FP64))
    rng = np.random.default_rng(7 + m)
    rows = np.unique(np.concatenate([rng.choice(ns.n_nodes, size=300, replace=False),
                                     [0, 999, ns.n_nodes - 1], np.arange(ns.n_nodes - 40, ns.n_nodes)]))
    full = np.zeros_like(nbr)
    full[rows] = nbr[rows]
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, full, m=m, n=n, rows=rows,
                                              form=FORM[m])
    w64, _ = oracle.weights(ns.x, ns.y, full, m=m, n=n, rows=rows)
    check_mixed(w[rows], st[rows], it[rows], w_mx, st_mx, it_mx, w64, n, exact=m == 2,
                what=f"1M m={m}")
    say("  statuses", np.bincount(st), "mean corrections", it[st == 0].mean())


@pytest.mark.parametrize("i,k,tries", [(40, 16, 1), (90, 7, 1), (40, 8, 10), (90, 1, 10)])
def test_mixed_fallback_rule_and_cap(i, k, tries):
    """The crafted stencils of the oracle's fallback pins (corrections that
    shrink by more or less than one half, or too slowly for the cap): the
    GPU falls back at the same correction."""
    ns = nodes.unit_square(12, seed=3)
    nbr = oracle.knn(ns.x, ns.y, 12)
    d = 10.0 ** (-4.0 - k / 20.0)
    x, y = ns.x.copy(), ns.y.copy()
    x[nbr[i, 4]] = x[nbr[i, 3]] + d
    y[nbr[i, 4]] = y[nbr[i, 3]] + 0.3 * d
    w_mx, st_mx, it_mx = oracle.weights_mixed(x, y, nbr, m=2, n=12)
    w, st, it = gpu_mixed(x, y, nbr, m=2, n=12)
    assert st_mx[i] == oracle.FELL_BACK and it_mx[i] == tries
    assert np.array_equal(st, st_mx) and np.array_equal(it, it_mx)
    assert rel_err(w, w_mx, 12).max() <= 1e-12


@pytest.mark.parametrize("m", [4, 6])
def test_mixed_blocked_fallback_and_failures(m):
    """The matrix-core mixed kernels: an ill-conditioned stencil (two support
    nodes 1e-6 h apart) falls back to FP64 on both sides and gets the FP64
    weights; a duplicate node and a bad index fail without fallback; the
    rest refine."""
    n = NFM[m]
    ns = nodes.unit_square(14, seed=5)
    nbr = oracle.knn(ns.x, ns.y, n)
    x, y = ns.x.copy(), ns.y.copy()
    i = 100
    x[nbr[i, 6]] = x[nbr[i, 5]] + 1e-6 / 14
    y[nbr[i, 6]] = y[nbr[i, 5]]
    nb = nbr.copy()
    nb[20, 5] = nb[20, 4]
    nb[21, 2] = 10 ** 6
    w_mx, st_mx, it_mx = oracle.weights_mixed(x, y, nb, m=m, n=n, form=oracle.MIXED_GJ)
    w64, _ = oracle.weights(x, y, nb, m=m, n=n)
    w, st, it = gpu_mixed(x, y, nb, m=m, n=n)
    say(f"m={m}: oracle statuses {np.bincount(st_mx)}, gpu {np.bincount(st)}")
    assert st_mx[20] == oracle.DUPLICATE and st_mx[21] == oracle.BAD_INDEX
    assert st_mx[i] == oracle.FELL_BACK
    check_mixed(w, st, it, w_mx, st_mx, it_mx, w64, n, exact=False, what=f"fallback m={m}")
    assert np.array_equal(w[i, :n], w64[i, :n])  # the FP64 kernel's weights, bit for bit


@pytest.mark.parametrize("op,oop", [(rb.OP_DX, oracle.D_DX), (rb.OP_DY, oracle.D_DY)],
                         ids=["dx", "dy"])
@pytest.mark.parametrize("m", [2, 4, 6])
def test_mixed_derivatives(m, op, oop):
    """The derivative operators in mixed precision (rbffd_weights_op_mixed)
    against the oracle's mixed form of the same operator and its FP64
    derivative weights, as the Laplacian above."""
    ns = nodes.unit_disk(3000, 200, seed=22)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n, form=FORM[m], op=oop)
    w64, _ = oracle.weights_op(ns.x, ns.y, nbr, m, n, oop)
    it = torch.zeros(ns.n_nodes, dtype=torch.int32, device="cuda")
    w, st = rb.rbffd_weights_op_mixed(dev(ns.x), dev(ns.y), dev(nbr), m, n, op, refine_steps=it)
    w, st, it = host(w), host(st), host(it)
    say("mixed derivative", m, op, "statuses", np.bincount(st), "mean corrections",
        it[st == 0].mean())
    check_mixed(w, st, it, w_mx, st_mx, it_mx, w64, n, exact=m == 2, what=f"op {op} m={m}")


def test_mixed_derivatives_full_size_and_errors():
    """The 1M-node square at m = 6, d/dx: sampled rows against the oracle's
    mixed form; unsupported supports and bad operators are refused."""
    ns = nodes.workload("square_1m_m6")
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, 56)
    it = torch.zeros(ns.n_nodes, dtype=torch.int32, device="cuda")
    w, st = rb.rbffd_weights_op_mixed(X, Y, NB, 6, 56, rb.OP_DX, refine_steps=it)
    w, st, it, nbr = host(w), host(st), host(it), host(NB)
    assert np.all((st == 0) | (st == rb.FELL_BACK_FP64))
    rows = np.unique(np.concatenate([np.random.default_rng(23).choice(ns.n_nodes, 150, replace=False),
                                     [0, ns.n_nodes - 1]]))
    full = np.zeros_like(nbr)
    full[rows] = nbr[rows]
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, full, m=6, n=56, rows=rows,
                                              form=oracle.MIXED_GJ, op=oracle.D_DX)
    w64, _ = oracle.weights_op(ns.x, ns.y, full, 6, 56, oracle.D_DX, rows=rows)
    check_mixed(w[rows], st[rows], it[rows], w_mx, st_mx, it_mx, w64, 56, exact=False,
                what="1M d/dx m=6")
    with pytest.raises(rb.RbffdError):  # a non-standard support
        rb.rbffd_weights_op_mixed(X[:1000], Y[:1000], NB[:1000, :40].contiguous(), 6, 40,
                                  rb.OP_DX)
    with pytest.raises(rb.RbffdError):  # the Laplacian's mixed form is rbffd_weights
        rb.rbffd_weights_op_mixed(X, Y, NB, 6, 56, rb.OP_LAPLACIAN)
