"""GPU explicit pseudo-time loop (eq. (3)) against the oracle's loop, bit for
bit: the same fma order per node and the same two roundings per update."""

import numpy as np
import pytest
import torch

import oracle
from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


def _problem(ns, m, n):
    nbr = oracle.knn(ns.x, ns.y, n)
    w, st = oracle.weights(ns.x, ns.y, nbr, m=m, n=n)
    assert np.all(st == 0)
    u_exact, F = nodes.manufactured(ns.x, ns.y)
    f = -F
    u0 = np.where(ns.is_boundary != 0, u_exact, 0.0)
    return nbr, w, f, u0


@pytest.mark.parametrize("steps", [0, 1, 2, 7, 33])
def test_time_loop_bit_exact_square_m2(steps):
    ns = nodes.workload("square_h45_m2")
    nbr, w, f, u0 = _problem(ns, 2, 12)
    dt = 1e-4
    ref = oracle.time_steps(nbr, w, 12, f, u0, dt, steps, is_boundary=ns.is_boundary)
    u = dev(u0)
    rb.rbffd_time_steps(dev(nbr), dev(w), 12, dev(f), u, dt, steps, is_boundary=dev(ns.is_boundary))
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref)


def test_time_loop_bit_exact_disk_m4_padded_stride():
    ns = nodes.unit_disk(3000, 200, seed=12)
    nbr, w, f, u0 = _problem(ns, 4, 30)
    # rows padded to a stride of 34 columns (the loop reads the first n)
    nbr_p = np.concatenate([nbr, np.zeros((ns.n_nodes, 4), np.int32)], axis=1)
    w_p = np.concatenate([w, np.full((ns.n_nodes, 4), np.nan)], axis=1)
    ref = oracle.time_steps(nbr_p, w_p, 30, f, u0, 1e-6, 11, is_boundary=ns.is_boundary)
    u = dev(u0)
    rb.rbffd_time_steps(dev(nbr_p), dev(w_p), 30, dev(f), u, 1e-6, 11,
                        is_boundary=dev(ns.is_boundary))
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref)


def test_time_loop_full_size_disk():
    """101k-node disk, m = 4, GPU supports and weights (bit-exact with the
    oracle's by the other parity tests), 50 steps: the whole state against
    the oracle's loop."""
    ns = nodes.workload("disk_100k_m4")
    X, Y = dev(ns.x), dev(ns.y)
    NB = rb.rbffd_knn(X, Y, 30)
    W, st, _ = rb.rbffd_weights(X, Y, NB, m=4, n=30)
    assert int((st != 0).sum()) == 0
    u_exact, F = nodes.manufactured(ns.x, ns.y)
    f = -F
    u0 = np.where(ns.is_boundary != 0, u_exact, 0.0)
    ref = oracle.time_steps(NB.cpu().numpy(), W.cpu().numpy(), 30, f, u0, 1e-6, 50,
                            is_boundary=ns.is_boundary)
    u = dev(u0)
    rb.rbffd_time_steps(NB, W, 30, dev(f), u, 1e-6, 50, is_boundary=dev(ns.is_boundary))
    torch.cuda.synchronize()
    assert np.array_equal(u.cpu().numpy(), ref)


def test_time_loop_bad_index_and_errors():
    ns = nodes.workload("square_h45_m2")
    nbr, w, f, u0 = _problem(ns, 2, 12)
    i = int(np.nonzero(ns.is_boundary == 0)[0][5])
    nb = nbr.copy()
    nb[i, 3] = -1
    ref = oracle.time_steps(nb, w, 12, f, u0, 1e-4, 2, is_boundary=ns.is_boundary)
    u = dev(u0)
    rb.rbffd_time_steps(dev(nb), dev(w), 12, dev(f), u, 1e-4, 2, is_boundary=dev(ns.is_boundary))
    got = u.cpu().numpy()
    assert np.isnan(got[i]) and np.array_equal(np.isnan(got), np.isnan(ref))
    assert np.array_equal(got[~np.isnan(got)], ref[~np.isnan(ref)])
    with pytest.raises(rb.RbffdError):
        rb.rbffd_time_steps(dev(nbr), dev(w), 13, dev(f), dev(u0), 1e-4, 1)
    with pytest.raises(rb.RbffdError):
        rb.rbffd_time_steps(dev(nbr), dev(w), 12, dev(f), dev(u0), 1e-4, -1)


@pytest.mark.parametrize("n_target", [30000, 40000])
def test_time_loop_bit_exact_mid_size(n_target):
    """Mid-size node sets (30k, 40k), an even and an odd number of steps (the
    result ends in either buffer): the same bits as the oracle's loop."""
    ns = nodes.unit_disk(n_target, 600, seed=13)
    nbr, w, f, u0 = _problem(ns, 2, 12)
    for steps in (8, 9):
        ref = oracle.time_steps(nbr, w, 12, f, u0, 1e-6, steps, is_boundary=ns.is_boundary)
        u = dev(u0)
        rb.rbffd_time_steps(dev(nbr), dev(w), 12, dev(f), u, 1e-6, steps,
                            is_boundary=dev(ns.is_boundary))
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref), f"N={ns.n_nodes} steps={steps}"


def test_time_loop_graph_replay():
    """The step loop captured in a graph: every replay (u reset eagerly
    between replays) gives the oracle's bits."""
    ns = nodes.unit_disk(3000, 200, seed=14)
    nbr, w, f, u0 = _problem(ns, 2, 12)
    steps = 7
    ref = oracle.time_steps(nbr, w, 12, f, u0, 1e-6, steps, is_boundary=ns.is_boundary)
    NB, W, F, B = dev(nbr), dev(w), dev(f), dev(ns.is_boundary)
    U0 = dev(u0)
    u = U0.clone()
    work = torch.empty_like(u)
    ws = torch.empty(ns.n_nodes * 12 * 12 + 1024, dtype=torch.uint8, device="cuda")

    def run():
        rb.rbffd_time_steps(NB, W, 12, F, u, 1e-6, steps, is_boundary=B, u_work=work,
                            workspace=ws)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        u.copy_(U0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(u.cpu().numpy(), ref), rep
