"""The C-ABI library loads on a machine without a GPU and exports every
function that include/rbffd.h declares.  No compute call is made here."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rbffd.h")
LIB = os.path.join(ROOT, "paper_2107_03632_amd", "librbffd.so")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rbffd_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("librbffd.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for fn in ["rbffd_knn", "rbffd_weights", "rbffd_weights_backward", "rbffd_assemble_csr",
               "rbffd_spmv", "rbffd_time_steps", "rbffd_solve", "rbffd_weights_op",
               "rbffd_knn3_workspace_size", "rbffd_knn3", "rbffd_weights3", "rbffd_weights3_op",
               "rbffd_weights3_batch_workspace_size", "rbffd_weights3_batch",
               "rbffd_weights_op_batch_workspace_size", "rbffd_weights_op_batch",
               "rbffd_weights_op_mixed_workspace_size", "rbffd_weights_op_mixed"]:
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(rbffd_\w+)$", out, flags=re.M))
    missing = [n for n in declared() if n not in exported]
    assert not missing, missing
    for n in declared():
        getattr(lib, n)


def test_host_only_queries(lib):
    lib.rbffd_error_string.restype = ctypes.c_char_p
    assert b"invalid" in lib.rbffd_error_string(-1)
    assert lib.rbffd_version() >= 100
    sz = ctypes.c_size_t(0)
    lib.rbffd_knn_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32,
                                             ctypes.POINTER(ctypes.c_size_t)]
    assert lib.rbffd_knn_workspace_size(100000, 30, ctypes.byref(sz)) == 0
    assert sz.value > 100000 * 24
    assert lib.rbffd_knn_workspace_size(10, 30, ctypes.byref(sz)) == -1  # k > n
    lib.rbffd_weights_save_size.argtypes = [ctypes.c_int64, ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_size_t)]
    assert lib.rbffd_weights_save_size(1000, 45, ctypes.byref(sz)) == 0
    assert sz.value >= 1000 * (8 * 45 * 45 + 8 * 45 + 8 + 45)


def test_argument_errors_before_any_launch(lib):
    # null pointers are rejected on the host, so no device is touched
    P = ctypes.c_void_p
    lib.rbffd_spmv.argtypes = [ctypes.c_int64, P, P, P, P, P, P, P]
    assert lib.rbffd_spmv(10, None, None, None, None, None, None, None) == -1
    lib.rbffd_knn.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P]
    assert lib.rbffd_knn(None, None, 10, 3, None, None, 0, None) == -1
    lib.rbffd_time_steps.argtypes = [ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32, P, P, P,
                                     ctypes.c_double, ctypes.c_int64, P, P, P, ctypes.c_size_t, P]
    assert lib.rbffd_time_steps(10, None, 12, 12, None, None, None, 1e-3, 1, None, None,
                                None, 0, None) == -1
    I32P, DP = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
    lib.rbffd_solve.argtypes = [ctypes.c_int64, P, P, P, P, P, ctypes.c_double, ctypes.c_int32,
                                I32P, DP, I32P, P, ctypes.c_size_t, P]
    it, rr, info = ctypes.c_int32(), ctypes.c_double(), ctypes.c_int32()
    assert lib.rbffd_solve(10, None, None, None, None, None, 1e-10, 100, ctypes.byref(it),
                           ctypes.byref(rr), ctypes.byref(info), None, 0, None) == -1
    lib.rbffd_weights_op.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_int32, ctypes.c_int32, P, P, P]
    assert lib.rbffd_weights_op(None, None, 10, None, 12, 2, 12, 1, None, None, None) == -1
    lib.rbffd_weights3.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, P, P, P]
    assert lib.rbffd_weights3(None, None, None, 10, None, 20, 2, 20, None, None, None) == -1
    lib.rbffd_weights3_op.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.c_int32, P, P, P]
    assert lib.rbffd_weights3_op(None, None, None, 10, None, 20, 2, 20, 1, None, None,
                                 None) == -1
    lib.rbffd_knn3.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_size_t, P]
    assert lib.rbffd_knn3(None, None, None, 10, 5, None, None, 0, None) == -1
    lib.rbffd_knn3_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int32,
                                              ctypes.POINTER(ctypes.c_size_t)]
    sz3 = ctypes.c_size_t(0)
    assert lib.rbffd_knn3_workspace_size(1000, 20, ctypes.byref(sz3)) == 0 and sz3.value > 0
    assert lib.rbffd_knn3_workspace_size(1000, 128, ctypes.byref(sz3)) == 0
    assert lib.rbffd_knn3_workspace_size(1000, 129, ctypes.byref(sz3)) == -1
    lib.rbffd_weights3_batch.argtypes = [P, P, P, ctypes.c_int64, P, ctypes.c_int32, P, P, P,
                                         P, ctypes.c_size_t, P]
    assert lib.rbffd_weights3_batch(None, None, None, 10, None, 70, None, None, None, None, 0,
                                    None) == -1
    lib.rbffd_weights3_batch_workspace_size.argtypes = [ctypes.c_int64,
                                                        ctypes.POINTER(ctypes.c_size_t)]
    assert lib.rbffd_weights3_batch_workspace_size(1000, ctypes.byref(sz3)) == 0
    assert sz3.value >= 2 * 1000 * 4
    assert lib.rbffd_weights3_batch_workspace_size(0, ctypes.byref(sz3)) == -1
    lib.rbffd_weights_op_batch.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32, P,
                                           ctypes.c_int32, P, P, P, ctypes.c_size_t, P]
    assert lib.rbffd_weights_op_batch(None, None, 10, None, 56, None, 1, None, None, None, 0,
                                      None) == -1
    lib.rbffd_weights_op_mixed.argtypes = [P, P, ctypes.c_int64, P, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P, P,
                                           P, P, ctypes.c_size_t, P]
    assert lib.rbffd_weights_op_mixed(None, None, 10, None, 30, 4, 30, 1, None, None, None,
                                      None, 0, None) == -1
    sz = ctypes.c_size_t(0)
    lib.rbffd_solve_workspace_size.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
    assert lib.rbffd_solve_workspace_size(1000, ctypes.byref(sz)) == 0
    assert sz.value >= 6 * 1000 * 8
    assert lib.rbffd_solve_workspace_size(0, ctypes.byref(sz)) == -1


def test_noalloc_knn_refuses_on_the_host(lib):
    # argument errors and inputs past the fixed scratch are refused before
    # the device is touched (the pointers are never dereferenced)
    P = ctypes.c_void_p
    lib.rbffd_knn_noalloc.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, P, P]
    assert lib.rbffd_knn_noalloc(None, None, 10, 3, None, None) == -1
    fake = P(256)
    assert lib.rbffd_knn_noalloc(fake, fake, 100, 65, fake, None) == -3
    assert lib.rbffd_knn_noalloc(fake, fake, 3_000_000, 12, fake, None) == -4
    assert lib.rbffd_knn_noalloc(fake, fake, 1_400_000, 1, fake, None) == -4
    lib.rbffd_error_string.restype = ctypes.c_char_p
    assert b"no-allocation" in lib.rbffd_error_string(-4)


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2107_03632_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f
                assert "liboracle" not in txt, f
