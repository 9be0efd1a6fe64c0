"""GPU mixed-precision weights (FP32 factorisation + FP64 refinement,
FP64 fallback) against the oracle's mixed form and the FP64 oracle.

The GPU performs the same operations in the same precisions as the oracle's
mixed form (FP32 factorisation and solves with fused updates, FP64 fused
residuals), so weights, statuses (including fall-backs) and correction counts
are compared exactly; against the FP64 oracle the bar is 1e-9 relative per
stencil.
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
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, nbr, m=m, n=n)
    w64, st64 = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    w, st, it = gpu_mixed(ns.x, ns.y, nbr, m=m, n=n)
    say("mixed", m, "statuses", np.bincount(st), "mean corrections", it[st == 0].mean())
    assert np.array_equal(st, st_mx)
    assert np.array_equal(it, it_mx)
    e_mx = rel_err(w, w_mx, n)
    say(f"  vs mixed oracle {e_mx.max():.3e}, bit-exact {np.mean(e_mx == 0):.4f}")
    assert e_mx.max() <= 1e-12
    e64 = rel_err(w, w64, n)
    say(f"  vs FP64 oracle {e64.max():.3e}")
    assert e64.max() <= 1e-9


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
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, full, m=6, n=56, rows=rows)
    assert np.array_equal(st[rows], st_mx) and np.array_equal(it[rows], it_mx)
    assert rel_err(w[rows], w_mx, 56).max() <= 1e-12
    w64, _ = oracle.weights(ns.x, ns.y, full, m=6, n=56, rows=rows)
    assert rel_err(w[rows], w64, 56).max() <= 1e-9
    say("  statuses", np.bincount(st), "mean corrections", it[st == 0].mean())


def test_mixed_order_batch():
    ns = nodes.cell_centred_square(40, seed=3, order_seed=33)
    nbr = oracle.knn(ns.x, ns.y, 56)
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, nbr, order=ns.order)
    w, st, it = gpu_mixed(ns.x, ns.y, nbr, order=dev(ns.order))
    assert np.array_equal(st, st_mx) and np.array_equal(it, it_mx)
    for m in (2, 4, 6):
        sel = ns.order == m
        assert rel_err(w[sel], w_mx[sel], NFM[m]).max() <= 1e-12


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
    w_mx, st_mx, it_mx = oracle.weights_mixed(ns.x, ns.y, full, m=m, n=n, rows=rows)
    assert np.array_equal(st[rows], st_mx) and np.array_equal(it[rows], it_mx)
    assert rel_err(w[rows], w_mx, n).max() <= 1e-12
    w64, _ = oracle.weights(ns.x, ns.y, full, m=m, n=n, rows=rows)
    assert rel_err(w[rows], w64, n).max() <= 1e-9
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
