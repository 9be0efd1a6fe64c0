"""Mixed-order batch: the persistent one-launch path, its tuning knobs, and
the whole pipeline (kNN -> weights -> CSR -> W u - f) captured in a graph.

Every tuning setting must give the same bits (tuning changes speed only);
graph replays, interleaved with eager work, must reproduce the eager outputs
bit for bit.
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


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module", autouse=True)
def need_gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    rb.library_path()


def test_batch_tuning_changes_nothing_but_speed():
    ns = nodes.cell_centred_square(80, seed=3, order_seed=33)
    nbr = oracle.knn(ns.x, ns.y, 56)
    X, Y, NB, O = dev(ns.x), dev(ns.y), dev(nbr), dev(ns.order)
    saved = rb.batch_tuning_get()
    outs = []
    try:
        for bpc, gpt, po, obpc in [(1, [1, 1, 1], 0, [12, 16, 4]), (2, [4, 2, 2], 0, [1, 1, 1]),
                                   (4, [2, 1, 2], 0, [12, 16, 4]), (3, [1, 2, 1], 0, [12, 16, 4]),
                                   (2, [1, 1, 1], 1, [12, 16, 4]), (2, [1, 1, 1], 1, [1, 1, 1]),
                                   (2, [1, 1, 1], 1, [64, 3, 7]), (2, [1, 1, 1], 2, [12, 16, 4])]:
            rb.batch_tuning_set(bpc, gpt, po, obpc)
            assert rb.batch_tuning_get() == {"blocks_per_cu": bpc, "groups_per_tile": gpt,
                                             "per_order": po, "order_blocks_per_cu": obpc}
            w, st, _ = rb.rbffd_weights(X, Y, NB, order=O)
            torch.cuda.synchronize()
            outs.append((w.cpu().numpy(), st.cpu().numpy()))
    finally:
        rb.batch_tuning_set(saved["blocks_per_cu"], saved["groups_per_tile"],
                            saved["per_order"], saved["order_blocks_per_cu"])
    for w, st in outs[1:]:
        assert np.array_equal(w, outs[0][0]) and np.array_equal(st, outs[0][1])
    w_ref, st_ref = oracle.weights(ns.x, ns.y, nbr, order=ns.order)
    assert np.array_equal(outs[0][1], st_ref)
    for m in (2, 4, 6):
        sel = ns.order == m
        e = np.abs(outs[0][0][sel] - w_ref[sel]).max(1) / np.abs(w_ref[sel]).max(1)
        assert e.max() <= 1e-11
    with pytest.raises(rb.RbffdError):
        rb.batch_tuning_set(0, [1, 1, 1])
    with pytest.raises(rb.RbffdError):
        rb.batch_tuning_set(2, [1, 1, 1], 3)
    with pytest.raises(rb.RbffdError):
        rb.batch_tuning_set(2, [1, 1, 1], 1, [1, 65, 1])
    assert rb.batch_tuning_get() == saved


@pytest.fixture(params=[0, 1, 2], ids=["one_launch", "per_order", "per_order_blocks"])
def batch_form(request):
    saved = rb.batch_tuning_get()
    rb.batch_tuning_set(saved["blocks_per_cu"], saved["groups_per_tile"], request.param,
                        saved["order_blocks_per_cu"])
    yield request.param
    rb.batch_tuning_set(saved["blocks_per_cu"], saved["groups_per_tile"], saved["per_order"],
                        saved["order_blocks_per_cu"])


def test_pipeline_graph_capture_and_replay(batch_form):
    ns = nodes.cell_centred_square(100, seed=3, order_seed=33)
    X, Y, O = dev(ns.x), dev(ns.y), dev(ns.order)
    B = dev((np.arange(ns.n_nodes) % 23 == 0).astype(np.uint8))
    u, f = nodes.manufactured(ns.x, ns.y)
    U, F = dev(u), dev(f)

    def pipeline():
        nbr = rb.rbffd_knn(X, Y, 56)
        w, st, _ = rb.rbffd_weights(X, Y, nbr, order=O)
        rp, col, val = rb.rbffd_assemble_csr(nbr, w, order=O, is_boundary=B)
        r = rb.rbffd_spmv(rp, col, val, U, F)
        return nbr, w, st, rp, col, val, r

    eager = [t.clone() for t in pipeline()]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pipeline()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        captured = pipeline()
    names = ("nbr", "w", "status", "row_ptr", "col", "val", "residual")
    nnz = int(eager[3][-1])

    def same(got, ref):
        # col/val have capacity N * max n; only the first row_ptr[N] are defined
        for name, a, b in zip(names, got, ref):
            if name in ("col", "val"):
                a, b = a[:nnz], b[:nnz]
            assert torch.equal(a, b), name
    for rep in range(3):
        other = pipeline()  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        same(captured, eager)
        same(other, eager)


def test_batch_full_size_sampled(batch_form):
    # the 1M-node mixed-order square in the launch the benchmark times: every
    # status clean, sampled rows equal to the oracle's weights bit for bit
    ns = nodes.workload("square_1m_mixed")
    X, Y, O = dev(ns.x), dev(ns.y), dev(ns.order)
    NB = rb.rbffd_knn(X, Y, 56)
    w, st, _ = rb.rbffd_weights(X, Y, NB, order=O)
    torch.cuda.synchronize()
    w, st, nbr = w.cpu().numpy(), st.cpu().numpy(), NB.cpu().numpy()
    del X, Y, O, NB
    print("mixed-order 1M: statuses", np.bincount(st), flush=True)
    assert np.all(st == 0)
    rows = np.unique(np.concatenate([np.arange(0, ns.n_nodes, 3331), [ns.n_nodes - 1]]))
    nbr_ref = oracle.knn(ns.x, ns.y, 56, queries=rows)
    assert np.array_equal(nbr[rows], nbr_ref)
    full = np.zeros((ns.n_nodes, 56), dtype=np.int32)
    full[rows] = nbr_ref
    w_ref, st_ref = oracle.weights(ns.x, ns.y, full, order=ns.order, rows=rows)
    assert np.all(st_ref == 0)
    assert np.array_equal(w[rows], w_ref)
    # zeros past each node's n
    for m in (2, 4, 6):
        sel = ns.order == m
        assert np.all(w[sel][:, NFM[m]:] == 0.0)


def _replay_matches(run, outs):
    """Capture run() in a graph, replay it three times with eager work
    between the replays, and check every replay against the eager result."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        run()  # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    ref = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for rep in range(3):
        for o in outs:
            o.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o.view(torch.int64) if o.dtype == torch.float64 else o,
                               r.view(torch.int64) if r.dtype == torch.float64 else r), rep


def test_operator_and_3d_batches_replay_in_a_graph():
    """rbffd_weights_op_batch and rbffd_weights3_batch enqueue everything
    on the stream (no host synchronisation) and replay bit-identically."""
    ns = nodes.unit_disk(4000, 200, seed=41)
    nbr = oracle.knn(ns.x, ns.y, 56)
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    O = dev(np.random.default_rng(42).choice(np.array([2, 4, 6], np.int8), ns.n_nodes))
    w = torch.empty((ns.n_nodes, 56), dtype=torch.float64, device="cuda")
    st = torch.empty(ns.n_nodes, dtype=torch.int32, device="cuda")
    _replay_matches(lambda: rb.rbffd_weights_op_batch(X, Y, NB, O, rb.OP_DY, out=w, status=st),
                    [w, st])
    x, y, z = nodes.jittered_cube(14, seed=43)
    X3, Y3, Z3 = dev(x), dev(y), dev(z)
    NB3 = rb.rbffd_knn3(X3, Y3, Z3, 70)
    O3 = dev(np.random.default_rng(44).choice(np.array([2, 4], np.int8), x.shape[0]))
    w3 = torch.empty((x.shape[0], 70), dtype=torch.float64, device="cuda")
    st3 = torch.empty(x.shape[0], dtype=torch.int32, device="cuda")
    _replay_matches(lambda: rb.rbffd_weights3_batch(X3, Y3, Z3, NB3, O3, out=w3, status=st3),
                    [w3, st3])


@pytest.mark.parametrize("m", [2, 4, 6])
def test_operator_batch_single_order(m):
    """Every node of one order (the other two lists empty): the batch gives
    rbffd_weights_op's weights at that order, bit for bit."""
    n = {2: 12, 4: 30, 6: 56}[m]
    ns = nodes.unit_disk(2000, 160, seed=45)
    nbr = oracle.knn(ns.x, ns.y, 56)
    X, Y, NB = dev(ns.x), dev(ns.y), dev(nbr)
    O = dev(np.full(ns.n_nodes, m, np.int8))
    w_b, st_b = rb.rbffd_weights_op_batch(X, Y, NB, O, rb.OP_DX)
    w_s, st_s = rb.rbffd_weights_op(X, Y, NB[:, :n].contiguous(), m, n, rb.OP_DX)
    assert torch.equal(st_b, st_s)
    assert torch.equal(w_b[:, :n], w_s) and torch.all(w_b[:, n:] == 0.0)
