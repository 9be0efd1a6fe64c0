"""The binding refuses mismatched shapes, dtypes and non-contiguous outputs
with an exception raised before any library call (a short coordinate or
vector array would otherwise be read past its end by the kernels)."""

import numpy as np
import pytest
import torch

from paper_2107_03632_amd import binding as rb
from paper_2107_03632_amd import nodes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible GPU")
    ns = nodes.unit_square(10, seed=3)
    X = torch.as_tensor(ns.x).cuda()
    Y = torch.as_tensor(ns.y).cuda()
    NB = rb.rbffd_knn(X, Y, 12)
    torch.cuda.synchronize()
    return ns, X, Y, NB


def test_knn_checks(case):
    ns, X, Y, NB = case
    with pytest.raises(ValueError):
        rb.rbffd_knn(X, Y[:-1], 12)
    with pytest.raises(ValueError):
        rb.rbffd_knn3(X, Y, Y[:-3], 12)
    with pytest.raises(ValueError):
        rb.rbffd_knn3(X, Y, Y, 12, out=torch.empty((X.numel(), 11), dtype=torch.int32,
                                                   device="cuda"))


def test_weights_checks(case):
    ns, X, Y, NB = case
    N = X.numel()
    with pytest.raises(ValueError):
        rb.rbffd_weights(X[:-1], Y, NB, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y[:5], NB, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y, NB[0], m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y, NB, order=torch.full((N - 1,), 2, dtype=torch.int8,
                                                    device="cuda"))
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y, NB, m=2, n=12,
                         out=torch.empty((N, 13), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):  # a non-contiguous output would be copied, not written
        rb.rbffd_weights(X, Y, NB, m=2, n=12,
                         out=torch.empty((12, N), dtype=torch.float64, device="cuda").t())
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y, NB, m=2, n=12,
                         status=torch.empty(N + 1, dtype=torch.int32, device="cuda"))
    with pytest.raises(ValueError):
        rb.rbffd_weights(X, Y, NB, m=2, n=12, precision=rb.MIXED,
                         refine_steps=torch.empty((N, 2), dtype=torch.int32, device="cuda")[:, 0])
    with pytest.raises(TypeError):
        rb.rbffd_weights(X, Y, NB, m=2, n=12,
                         status=torch.empty(N, dtype=torch.int64, device="cuda"))
    with pytest.raises(ValueError):
        rb.rbffd_weights_op(X, Y[:-2], NB, 2, 12, rb.OP_DX)
    with pytest.raises(ValueError):
        rb.rbffd_weights3(X, Y, Y[:-1], NB, m=2, n=10)


def test_backward_checks(case):
    ns, X, Y, NB = case
    N = X.numel()
    _, st, sv = rb.rbffd_weights(X, Y, NB, m=2, n=12, save=True)
    G = torch.zeros((N, 12), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        rb.rbffd_weights_backward(X, Y, NB, G[:, :11], sv, status=st, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights_backward(X[:-1], Y, NB, G, sv, status=st, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights_backward(X, Y, NB, G, sv[:100], status=st, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_weights_backward(X, Y, NB, G, sv, status=st[:-1], m=2, n=12)


def test_csr_spmv_solve_timeloop_checks(case):
    ns, X, Y, NB = case
    N = X.numel()
    w, st, _ = rb.rbffd_weights(X, Y, NB, m=2, n=12)
    with pytest.raises(ValueError):
        rb.rbffd_assemble_csr(NB, w[:, :11], n=12)
    with pytest.raises(ValueError):
        rb.rbffd_assemble_csr(NB, w, n=12, is_boundary=torch.zeros(N - 1, dtype=torch.uint8,
                                                                   device="cuda"))
    rp, col, val = rb.rbffd_assemble_csr(NB, w, n=12)
    u = torch.ones(N, dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        rb.rbffd_spmv(rp, col, val, u[:-1])
    with pytest.raises(ValueError):
        rb.rbffd_spmv(rp, col, val, u, f=u[:-1])
    with pytest.raises(ValueError):
        rb.rbffd_spmv(rp, col, val[:-1], u)
    with pytest.raises(ValueError):
        rb.rbffd_spmv(rp, col, val, u, out=torch.empty(N - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        rb.rbffd_solve(rp, col, val, u[:-1])
    with pytest.raises(ValueError):
        rb.rbffd_solve(rp, col, val, u, x0=u[:-2])
    with pytest.raises(ValueError):
        rb.rbffd_time_steps(NB, w, 12, u[:-1], u.clone(), 1e-6, 2)
    with pytest.raises(ValueError):
        rb.rbffd_time_steps(NB, w, 12, u, torch.ones(2 * N, dtype=torch.float64,
                                                       device="cuda")[::2], 1e-6, 2)
    # the correct calls still run
    y = rb.rbffd_spmv(rp, col, val, u)
    torch.cuda.synchronize()
    assert np.isfinite(y.cpu().numpy()).all()
