"""rbffd_knn_noalloc (the kNN entry point that allocates nothing and keeps
its scratch in a fixed device array of the library) against rbffd_knn on
the same inputs, through the C ABI: bit-exact supports on two calls in a
row, the second with a smaller input, so the second call runs on the first
call's leftover scratch; then a larger k and the oracle on a small set."""

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


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_noalloc_matches_knn_on_consecutive_calls():
    cases = [("disk_100k_m4", 30), ("square_h45_m2", 12), ("square_h45_m2", 56),
             ("disk_100k_m4", 12)]
    for name, k in cases:
        ns = nodes.workload(name)
        say("knn_noalloc", name, ns.n_nodes, "k =", k)
        X = torch.as_tensor(ns.x, device="cuda")
        Y = torch.as_tensor(ns.y, device="cuda")
        a = rb.rbffd_knn_noalloc(X, Y, k)
        b = rb.rbffd_knn(X, Y, k)
        assert np.array_equal(host(a), host(b)), f"{name} k={k}: differs from rbffd_knn"
        if ns.n_nodes < 5000:
            assert np.array_equal(host(a), oracle.knn(ns.x, ns.y, k))


def test_noalloc_output_in_place_and_limits():
    ns = nodes.workload("square_h45_m2")
    X = torch.as_tensor(ns.x, device="cuda")
    Y = torch.as_tensor(ns.y, device="cuda")
    out = torch.full((ns.n_nodes, 12), -7, dtype=torch.int32, device="cuda")
    r = rb.rbffd_knn_noalloc(X, Y, 12, out=out)
    assert r.data_ptr() == out.data_ptr()
    assert np.array_equal(host(out), oracle.knn(ns.x, ns.y, 12))
    # sizes past the fixed scratch are refused on the host, before any launch
    lib = rb._load()
    P = rb._p
    rc = lib.rbffd_knn_noalloc(P(X), P(Y), 3_000_000, 12, P(out),
                               rb._stream(X.device))
    assert rc == -4, rc
    assert "no-allocation" in rb.error_string(rc)
