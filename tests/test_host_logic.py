"""Host-side behaviour that needs no GPU: the bench refuses more than one GPU,
and the binding refuses CPU tensors before any library call."""

import os
import subprocess
import sys

import pytest
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2",
                        "--steps", "1", "--warmup", "0"], capture_output=True, text=True,
                       timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_binding_refuses_cpu_tensors():
    from paper_2107_03632_amd import binding as rb
    x = torch.zeros(10, dtype=torch.float64)
    with pytest.raises(rb.RbffdError, match="GPU tensor"):
        rb.rbffd_knn(x, x, 3)
    with pytest.raises(rb.RbffdError, match="GPU tensor"):
        rb.rbffd_knn3(x, x, x, 3)
    with pytest.raises(TypeError, match="torch tensor"):
        rb.rbffd_knn(x.numpy(), x.numpy(), 3)
