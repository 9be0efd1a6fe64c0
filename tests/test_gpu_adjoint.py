"""GPU adjoint (rbffd_weights_backward) against the oracle's adjoint and
against central finite differences, through the C ABI and through the
autograd wrapper.

Tolerances: the per-slot contributions follow the oracle's operation order;
only the order of the final per-node sums differs (the GPU gathers the
stencil's own term first, then the slots that name the node by index), so the
difference is a few rounding errors of the largest term: bound
max|g_gpu - g_ref| <= 1e-11 * max|g_ref|.  Finite differences: <= 1e-6
relative (step 1e-6 h two-point at m = 2, 4; 1e-4 h four-point at m = 6,
whose boundary stencils have cond ~1e7).
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
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


@pytest.mark.parametrize("m", [2, 4, 6])
def test_backward_matches_oracle_adjoint(m):
    say("adjoint vs oracle", m)
    ns = nodes.annulus(1500, seed=8)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    G = nodes.gaussian_cotangent(ns.n_nodes, n, seed=55)
    gx_ref, gy_ref, failed = oracle.adjoint(ns.x, ns.y, nbr, G, m=m, n=n)
    assert failed == 0
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    w, st, sv = rb.rbffd_weights(X, Y, NB, m=m, n=n, save=True)
    gx, gy = rb.rbffd_weights_backward(X, Y, NB, dev(G), sv, status=st, m=m, n=n)
    gx, gy = host(gx), host(gy)
    scale = max(np.abs(gx_ref).max(), np.abs(gy_ref).max())
    err = max(np.abs(gx - gx_ref).max(), np.abs(gy - gy_ref).max()) / scale
    say(f"  max rel err {err:.3e}")
    assert err <= 1e-11
    # deterministic: a second call gives the same bits
    gx2, gy2 = rb.rbffd_weights_backward(X, Y, NB, dev(G), sv, status=st, m=m, n=n)
    assert np.array_equal(host(gx2), gx) and np.array_equal(host(gy2), gy)


def _gpu_local_loss(X, Y, NB, G, m, n, rows):
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=m, n=n)
    assert int((st[rows] != 0).sum()) == 0
    return float((G[rows] * w[rows]).sum())


@pytest.mark.parametrize("m", [2, 4, 6])
def test_backward_matches_finite_differences(m):
    say("adjoint vs FD", m)
    ns = nodes.annulus(1500, seed=8)
    n = NFM[m]
    nbr = oracle.knn(ns.x, ns.y, n)
    G = dev(nodes.gaussian_cotangent(ns.n_nodes, n, seed=55))
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    _, st, sv = rb.rbffd_weights(X, Y, NB, m=m, n=n, save=True)
    gx, gy = rb.rbffd_weights_backward(X, Y, NB, G, sv, status=st, m=m, n=n)
    gx, gy = host(gx), host(gy)
    d = (1e-4 if m == 6 else 1e-6) * ns.h
    taps = ((2, -1 / 12), (1, 8 / 12), (-1, -8 / 12), (-2, 1 / 12)) if m == 6 \
        else ((1, 0.5), (-1, -0.5))
    rng = np.random.default_rng(2)
    adj, fd = [], []
    for p in rng.choice(ns.n_nodes, size=10, replace=False):
        rows = np.unique(np.concatenate([[p], np.nonzero(np.any(nbr == p, axis=1))[0]]))
        rows_t = torch.as_tensor(rows).cuda()
        for coord, g in ((0, gx), (1, gy)):
            acc = 0.0
            for sgn, c in taps:
                x, y = ns.x.copy(), ns.y.copy()
                (x if coord == 0 else y)[p] += sgn * d
                acc += c * _gpu_local_loss(dev(x), dev(y), NB, G, m, n, rows_t)
            fd.append(acc / d)
            adj.append(g[p])
    adj, fd = np.array(adj), np.array(fd)
    err = np.abs(adj - fd).max() / np.abs(fd).max()
    say(f"  FD rel err {err:.3e}")
    assert err <= 1e-6


def test_autograd_function_and_residual_loss():
    """L1 = sum g w and L2 = |W u - f|^2 (interior rows, u and f from the
    coordinates) through torch autograd; gradients checked by FD."""
    ns = nodes.unit_square(16, seed=6)
    n, m = 30, 4
    nbr = oracle.knn(ns.x, ns.y, n)
    NB = dev(nbr)
    inter = dev((ns.is_boundary == 0))

    def loss2(X, Y):
        w, st = rb.weights(X, Y, NB, m=m, n=n)
        u = torch.sin(np.pi * X) * torch.sin(np.pi * Y)
        f = -2 * np.pi ** 2 * u
        r = (w * u[NB.long()]).sum(1) - f
        return (r[inter] ** 2).sum()

    X = dev(ns.x).requires_grad_(True)
    Y = dev(ns.y).requires_grad_(True)
    L = loss2(X, Y)
    gx, gy = torch.autograd.grad(L, (X, Y))
    gx, gy = host(gx), host(gy)
    d = 1e-6 * ns.h
    for p in [3, 50, 120, ns.n_nodes - 1]:
        for coord, g in ((0, gx), (1, gy)):
            vals = []
            for sgn in (1, -1):
                x, y = ns.x.copy(), ns.y.copy()
                (x if coord == 0 else y)[p] += sgn * d
                vals.append(float(loss2(dev(x), dev(y))))
            fd = (vals[0] - vals[1]) / (2 * d)
            assert abs(fd - g[p]) <= 1e-6 * max(1.0, np.abs(gx).max(), np.abs(gy).max()), \
                (p, coord, fd, g[p])


def test_backward_mixed_order_matches_oracle():
    ns = nodes.cell_centred_square(40, seed=3, order_seed=33)
    say("adjoint mixed order", ns.n_nodes)
    nbr = oracle.knn(ns.x, ns.y, 56)
    G = nodes.gaussian_cotangent(ns.n_nodes, 56, seed=9)
    gx_ref, gy_ref, failed = oracle.adjoint(ns.x, ns.y, nbr, G, order=ns.order)
    assert failed == 0
    X, Y, NB, O = dev(ns.x), dev(ns.y), dev(nbr), dev(ns.order)
    _, st, sv = rb.rbffd_weights(X, Y, NB, order=O, save=True)
    gx, gy = rb.rbffd_weights_backward(X, Y, NB, dev(G), sv, status=st, order=O)
    scale = max(np.abs(gx_ref).max(), np.abs(gy_ref).max())
    err = max(np.abs(host(gx) - gx_ref).max(), np.abs(host(gy) - gy_ref).max()) / scale
    assert err <= 1e-11


def test_backward_full_size_annulus():
    """200k-node annulus, m = 4: zero net force (L depends on differences
    only) at full size, and finite differences on sampled coordinates."""
    ns = nodes.workload("annulus_200k_m4")
    say("adjoint annulus", ns.n_nodes)
    n, m = 30, 4
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, n)
    G = dev(nodes.gaussian_cotangent(ns.n_nodes, n, seed=55))
    _, st, sv = rb.rbffd_weights(X, Y, NB, m=m, n=n, save=True)
    assert int((st != 0).sum()) == 0
    gx, gy = rb.rbffd_weights_backward(X, Y, NB, G, sv, status=st, m=m, n=n)
    gx, gy = host(gx), host(gy)
    assert abs(gx.sum()) <= 1e-9 * np.abs(gx).sum()
    assert abs(gy.sum()) <= 1e-9 * np.abs(gy).sum()
    nbr = host(NB)
    d = 1e-6 * ns.h
    rng = np.random.default_rng(4)
    adj, fd = [], []
    for p in rng.choice(ns.n_nodes, size=6, replace=False):
        rows = np.unique(np.concatenate([[p], np.nonzero(np.any(nbr == p, axis=1))[0]]))
        rows_t = torch.as_tensor(rows).cuda()
        for coord, g in ((0, gx), (1, gy)):
            vals = []
            for sgn in (1, -1):
                x, y = ns.x.copy(), ns.y.copy()
                (x if coord == 0 else y)[p] += sgn * d
                vals.append(_gpu_local_loss(dev(x), dev(y), NB, G, m, n, rows_t))
            fd.append((vals[0] - vals[1]) / (2 * d))
            adj.append(g[p])
    err = np.abs(np.array(adj) - np.array(fd)).max() / np.abs(np.array(fd)).max()
    say(f"  FD rel err {err:.3e}")
    assert err <= 1e-6
    # the oracle's adjoint on 150 sampled nodes: every stencil that names a
    # sampled node (its own and those whose supports hold it) contributes
    sample = rng.choice(ns.n_nodes, size=150, replace=False)
    touch = np.nonzero(np.isin(nbr, sample).any(axis=1))[0]
    rows = np.unique(np.concatenate([sample, touch]))
    say(f"  oracle adjoint over {rows.size} stencils")
    gxo, gyo, failed = oracle.adjoint(ns.x, ns.y, nbr, host(G), m=m, n=n, rows=rows)
    assert failed == 0
    scale = max(np.abs(gxo[sample]).max(), np.abs(gyo[sample]).max())
    err = max(np.abs(gx[sample] - gxo[sample]).max(),
              np.abs(gy[sample] - gyo[sample]).max()) / scale
    say(f"  vs oracle adjoint {err:.3e}")
    assert err <= 1e-11
