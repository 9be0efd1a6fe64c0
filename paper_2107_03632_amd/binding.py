"""Python binding of librbffd.so: same names as the C ABI, torch tensors in.

Argument marshalling only.  Every step runs in the HIP library on the
caller's current torch stream; torch provides device memory (outputs and
workspaces) and the stream handle.  There is no CPU path: if the library is
missing or a tensor is not on the GPU, the call raises.
"""

from __future__ import annotations

import ctypes
import os
import threading

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librbffd.so")

FP64, MIXED = 0, 1
OK, SINGULAR, FELL_BACK_FP64, NONFINITE, BAD_INDEX, DUPLICATE, BAD_ORDER = range(7)
SOLVE_CONVERGED, SOLVE_MAX_ITER, SOLVE_BREAKDOWN, SOLVE_NONFINITE = range(4)
OP_LAPLACIAN, OP_DX, OP_DY, OP3_DZ = range(4)
DEFAULT_N_FOR_ORDER = (12, 30, 56)

_lock = threading.Lock()
_lib = None


class RbffdError(RuntimeError):
    pass


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RbffdError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
        PSZ = ctypes.POINTER(ctypes.c_size_t)
        sig = {
            "rbffd_error_string": ([ctypes.c_int], ctypes.c_char_p),
            "rbffd_version": ([], ctypes.c_int),
            "rbffd_knn_workspace_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_knn": ([P, P, I64, I32, P, P, SZ, P], ctypes.c_int),
            "rbffd_knn_noalloc": ([P, P, I64, I32, P, P], ctypes.c_int),
            "rbffd_weights_workspace_size": ([I64, I32, I32, PSZ], ctypes.c_int),
            "rbffd_weights_save_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_weights": ([P, P, I64, P, I32, P, I32, I32, P, I32, P, P, P, P, SZ, P, SZ,
                               P], ctypes.c_int),
            "rbffd_weights_backward_workspace_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_weights_backward": ([P, P, I64, P, I32, P, I32, I32, P, P, P, SZ, P, P, P,
                                        P, SZ, P], ctypes.c_int),
            "rbffd_assemble_csr_workspace_size": ([I64, PSZ], ctypes.c_int),
            "rbffd_assemble_csr": ([I64, P, I32, P, I32, P, P, P, P, P, P, I64, P, SZ, P],
                                   ctypes.c_int),
            "rbffd_spmv": ([I64, P, P, P, P, P, P, P], ctypes.c_int),
            "rbffd_time_steps_workspace_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_time_steps": ([I64, P, I32, I32, P, P, P, ctypes.c_double, I64, P, P, P, SZ,
                                  P], ctypes.c_int),
            "rbffd_weights_op": ([P, P, I64, P, I32, I32, I32, I32, P, P, P], ctypes.c_int),
            "rbffd_weights_op_batch_workspace_size": ([I64, PSZ], ctypes.c_int),
            "rbffd_weights_op_batch": ([P, P, I64, P, I32, P, I32, P, P, P, SZ, P], ctypes.c_int),
            "rbffd_weights_op_mixed_workspace_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_weights_op_mixed": ([P, P, I64, P, I32, I32, I32, I32, P, P, P, P, SZ, P],
                                       ctypes.c_int),
            "rbffd_knn3_workspace_size": ([I64, I32, PSZ], ctypes.c_int),
            "rbffd_knn3": ([P, P, P, I64, I32, P, P, ctypes.c_size_t, P], ctypes.c_int),
            "rbffd_weights3": ([P, P, P, I64, P, I32, I32, I32, P, P, P], ctypes.c_int),
            "rbffd_weights3_op": ([P, P, P, I64, P, I32, I32, I32, I32, P, P, P], ctypes.c_int),
            "rbffd_weights3_batch_workspace_size": ([I64, PSZ], ctypes.c_int),
            "rbffd_weights3_batch": ([P, P, P, I64, P, I32, P, P, P, P, SZ, P], ctypes.c_int),
            "rbffd_solve_workspace_size": ([I64, PSZ], ctypes.c_int),
            "rbffd_solve": ([I64, P, P, P, P, P, ctypes.c_double, I32,
                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_int32), P, SZ, P], ctypes.c_int),
            "rbffd_solve_async": ([I64, P, P, P, P, P, ctypes.c_double, I32, I32, P, P, SZ, P],
                                  ctypes.c_int),
            "rbffd_batch_tuning_set": ([P], ctypes.c_int),
            "rbffd_batch_tuning_get": ([P], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    _apply_saved_tuning()
    return lib


class BatchTuning(ctypes.Structure):
    _fields_ = [("blocks_per_cu", ctypes.c_int32), ("groups_per_tile", ctypes.c_int32 * 3),
                ("per_order", ctypes.c_int32), ("order_blocks_per_cu", ctypes.c_int32 * 3)]


TUNING_PATH = os.path.join(_HERE, "batch_tuning.json")
DEFAULT_ORDER_BLOCKS_PER_CU = (12, 16, 4)


def _tuning(blocks_per_cu, groups_per_tile, per_order=0,
            order_blocks_per_cu=DEFAULT_ORDER_BLOCKS_PER_CU) -> BatchTuning:
    i3 = ctypes.c_int32 * 3
    return BatchTuning(int(blocks_per_cu), i3(*[int(v) for v in groups_per_tile]),
                       int(per_order), i3(*[int(v) for v in order_blocks_per_cu]))


def batch_tuning_set(blocks_per_cu: int, groups_per_tile, per_order: int = 0,
                     order_blocks_per_cu=DEFAULT_ORDER_BLOCKS_PER_CU) -> None:
    """Set the mixed-order batch's form (one launch, or one launch per
    order) and its grid and tile sizes."""
    t = _tuning(blocks_per_cu, groups_per_tile, per_order, order_blocks_per_cu)
    _check(_load().rbffd_batch_tuning_set(ctypes.byref(t)), "rbffd_batch_tuning_set")


def batch_tuning_get() -> dict:
    t = BatchTuning()
    _check(_load().rbffd_batch_tuning_get(ctypes.byref(t)), "rbffd_batch_tuning_get")
    return {"blocks_per_cu": t.blocks_per_cu, "groups_per_tile": list(t.groups_per_tile),
            "per_order": t.per_order, "order_blocks_per_cu": list(t.order_blocks_per_cu)}


def _apply_saved_tuning():
    """Apply the autotuner's saved choice (batch_tuning.json), if any."""
    if not os.path.exists(TUNING_PATH):
        return
    import json
    with open(TUNING_PATH) as f:
        cfg = json.load(f)["choice"]
    t = _tuning(cfg["blocks_per_cu"], cfg["groups_per_tile"], cfg.get("per_order", 0),
                cfg.get("order_blocks_per_cu", DEFAULT_ORDER_BLOCKS_PER_CU))
    _check(_lib.rbffd_batch_tuning_set(ctypes.byref(t)), "rbffd_batch_tuning_set")


def library_path() -> str:
    _load()
    return LIB_PATH


def error_string(code: int) -> str:
    return _load().rbffd_error_string(code).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise RbffdError(f"{what} failed: {rc} ({error_string(rc)})")


def _dev(t: torch.Tensor, dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise RbffdError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    return t.contiguous()


def _vec(t: torch.Tensor, n: int, dtype, name: str) -> torch.Tensor:
    """An input of exactly n entries (the kernels index it by node or row)."""
    t = _dev(t, dtype, name)
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} entries, expected {n}")
    return t


def _supports(nbr: torch.Tensor) -> torch.Tensor:
    nbr = _dev(nbr, torch.int32, "nbr")
    if nbr.dim() != 2 or nbr.shape[1] < 1:
        raise ValueError(f"nbr must be [N, k], got shape {tuple(nbr.shape)}")
    return nbr


def _out(t, shape, dtype, name: str, device) -> torch.Tensor:
    """A caller-provided output: written in place, so it is never copied;
    anything but a contiguous device tensor of the exact shape is refused."""
    if t is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise RbffdError(f"{name} must be a GPU tensor (the library has no CPU path)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous (it is written in place)")
    return t


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _size(fn, *args) -> int:
    out = ctypes.c_size_t(0)
    _check(fn(*args, ctypes.byref(out)), fn.__name__)
    return int(out.value)


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _n_for_order(n_for_order):
    arr = (ctypes.c_int32 * 3)(*[int(v) for v in n_for_order])
    return arr


def n_monomials(m: int) -> int:
    return (m + 1) * (m + 2) // 2


# ---------------------------------------------------------------------------
def rbffd_knn(x: torch.Tensor, y: torch.Tensor, k: int) -> torch.Tensor:
    """k nearest nodes of every node, ascending by (d^2, index): int32 [N, k]."""
    lib = _load()
    x = _dev(x, torch.float64, "x")
    N = x.numel()
    y = _vec(y, N, torch.float64, "y")
    ws = _workspace(_size(lib.rbffd_knn_workspace_size, N, k), x.device)
    nbr = torch.empty((N, k), dtype=torch.int32, device=x.device)
    _check(lib.rbffd_knn(_p(x), _p(y), N, k, _p(nbr), _p(ws), ws.numel(), _stream(x.device)),
           "rbffd_knn")
    return nbr


def rbffd_knn_noalloc(x: torch.Tensor, y: torch.Tensor, k: int, out=None) -> torch.Tensor:
    """rbffd_knn with the library's fixed scratch instead of a workspace (the
    C call allocates nothing).  out: an optional int32 [N, k] output, written
    in place; without it one is allocated here, by torch."""
    lib = _load()
    x = _dev(x, torch.float64, "x")
    N = x.numel()
    y = _vec(y, N, torch.float64, "y")
    nbr = _out(out, (N, k), torch.int32, "out", x.device)
    _check(lib.rbffd_knn_noalloc(_p(x), _p(y), N, k, _p(nbr), _stream(x.device)),
           "rbffd_knn_noalloc")
    return nbr


def _order_args(order, m, n, n_for_order, N):
    if order is None:
        if m is None or n is None:
            raise ValueError("give (m, n) or a per-node order")
        return None, int(m), int(n), None, n + n_monomials(m)
    kmax = max(nv + n_monomials(mv) for mv, nv in zip((2, 4, 6), n_for_order))
    return _vec(order, N, torch.int8, "order"), -1, -1, _n_for_order(n_for_order), kmax


def _nodes2(x, y, nbr):
    """Coordinates and supports: x, y [N] FP64, nbr [N, k] int32."""
    nbr = _supports(nbr)
    N = nbr.shape[0]
    return _vec(x, N, torch.float64, "x"), _vec(y, N, torch.float64, "y"), nbr, N, nbr.shape[1]


def rbffd_weights(x, y, nbr, m=None, n=None, order=None, n_for_order=DEFAULT_N_FOR_ORDER,
                  precision: int = FP64, save: bool = False, out=None, status=None,
                  refine_steps=None):
    """Laplacian stencil weights w [N, k_stride] (FP64) and status [N] int32.

    Returns (w, status, save_buffer or None).  nbr is [N, k_stride] int32.
    precision=MIXED: FP32 factorisation + FP64 refinement; refine_steps (an
    int32 [N] tensor, optional) receives the corrections per stencil.
    """
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    o, m_, n_, nfo, kmax = _order_args(order, m, n, n_for_order, N)
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    sv = None
    if save:
        sv = _workspace(_size(lib.rbffd_weights_save_size, N, kmax), x.device)
    ws = _workspace(_size(lib.rbffd_weights_workspace_size, N, int(o is not None), precision),
                    x.device)
    rs = None if refine_steps is None else \
        _out(refine_steps, (N,), torch.int32, "refine_steps", x.device)
    _check(lib.rbffd_weights(_p(x), _p(y), N, _p(nbr), ks, _p(o), m_, n_, nfo, precision,
                             _p(w), _p(st), _p(rs), _p(sv), 0 if sv is None else sv.numel(),
                             _p(ws), ws.numel(), _stream(x.device)), "rbffd_weights")
    return w, st, sv


def rbffd_weights_op(x, y, nbr, m: int, n: int, op: int, out=None, status=None):
    """Weights of eq. (1) for the operator op (OP_LAPLACIAN, OP_DX, OP_DY),
    FP64, uniform (m, n).  Returns (w [N, k_stride], status [N])."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    _check(lib.rbffd_weights_op(_p(x), _p(y), N, _p(nbr), ks, int(m), int(n), int(op), _p(w),
                                _p(st), _stream(x.device)), "rbffd_weights_op")
    return w, st


def rbffd_knn3(x, y, z, k: int, out=None):
    """Supports of nodes in R^3: nbr [N, k] int32 (self first, ascending
    (d^2, index))."""
    lib = _load()
    x = _dev(x, torch.float64, "x")
    y = _dev(y, torch.float64, "y")
    z = _dev(z, torch.float64, "z")
    N = x.numel()
    y = _vec(y, N, torch.float64, "y")
    z = _vec(z, N, torch.float64, "z")
    ws = _workspace(_size(lib.rbffd_knn3_workspace_size, N, int(k)), x.device)
    nbr = _out(out, (N, int(k)), torch.int32, "out", x.device)
    _check(lib.rbffd_knn3(_p(x), _p(y), _p(z), N, int(k), _p(nbr), _p(ws), ws.numel(),
                          _stream(x.device)), "rbffd_knn3")
    return nbr


def rbffd_weights3(x, y, z, nbr, m: int = 2, n: int = 20, out=None, status=None, op=None):
    """Weights of eq. (1) for nodes in R^3 (r^3 + monomials of degree <= m,
    m = 2 with 10 <= n <= 54, or m = 4 with 35 <= n <= 76), FP64: the
    Laplacian, or with op one of OP_DX, OP_DY, OP3_DZ a first derivative.
    Returns (w [N, k_stride], status [N])."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    z = _vec(z, N, torch.float64, "z")
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    if op is None:
        _check(lib.rbffd_weights3(_p(x), _p(y), _p(z), N, _p(nbr), ks, int(m), int(n), _p(w),
                                  _p(st), _stream(x.device)), "rbffd_weights3")
    else:
        _check(lib.rbffd_weights3_op(_p(x), _p(y), _p(z), N, _p(nbr), ks, int(m), int(n),
                                     int(op), _p(w), _p(st), _stream(x.device)),
               "rbffd_weights3_op")
    return w, st


def rbffd_weights_op_mixed(x, y, nbr, m: int, n: int, op: int, out=None, status=None,
                           refine_steps=None):
    """d/dx (OP_DX) or d/dy (OP_DY) weights in mixed precision (FP32
    factorisation + FP64 refinement, FP64 fallback) on the standard
    supports.  refine_steps: an int32 [N] device tensor that receives the
    corrections per stencil.  Returns (w [N, k_stride], status [N])."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    it = None if refine_steps is None else _out(refine_steps, (N,), torch.int32,
                                                 "refine_steps", x.device)
    ws = _workspace(_size(lib.rbffd_weights_op_mixed_workspace_size, N, int(m)), x.device)
    _check(lib.rbffd_weights_op_mixed(_p(x), _p(y), N, _p(nbr), ks, int(m), int(n), int(op),
                                      _p(w), _p(st), _p(it), _p(ws), ws.numel(),
                                      _stream(x.device)), "rbffd_weights_op_mixed")
    return w, st


def rbffd_weights_op_batch(x, y, nbr, order, op: int, out=None, status=None):
    """d/dx (OP_DX) or d/dy (OP_DY) weights for a per-node order (int8 [N],
    2, 4 or 6) on the supports n = 12 / 30 / 56: nbr [N, k_stride] with
    k_stride >= 56.  Each node's weights and status are rbffd_weights_op's at
    its order.  Returns (w [N, k_stride], status [N])."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    order = _vec(order, N, torch.int8, "order")
    if ks < 56:
        raise ValueError(f"nbr needs at least 56 columns for the m = 6 class, got {ks}")
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    ws = _workspace(_size(lib.rbffd_weights_op_batch_workspace_size, N), x.device)
    _check(lib.rbffd_weights_op_batch(_p(x), _p(y), N, _p(nbr), ks, _p(order), int(op), _p(w),
                                      _p(st), _p(ws), ws.numel(), _stream(x.device)),
           "rbffd_weights_op_batch")
    return w, st


def rbffd_weights3_batch(x, y, z, nbr, order, out=None, status=None):
    """3-D Laplacian weights for a per-node order (int8 [N], 2 or 4) on the
    supports n = 20 / 70: nbr [N, k_stride] with k_stride >= 70.  Each
    node's weights and status are rbffd_weights3's at its order.
    Returns (w [N, k_stride], status [N])."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    z = _vec(z, N, torch.float64, "z")
    order = _vec(order, N, torch.int8, "order")
    if ks < 70:
        raise ValueError(f"nbr needs at least 70 columns for the m = 4 class, got {ks}")
    w = _out(out, (N, ks), torch.float64, "out", x.device)
    st = _out(status, (N,), torch.int32, "status", x.device)
    ws = _workspace(_size(lib.rbffd_weights3_batch_workspace_size, N), x.device)
    _check(lib.rbffd_weights3_batch(_p(x), _p(y), _p(z), N, _p(nbr), ks, _p(order), _p(w),
                                    _p(st), _p(ws), ws.numel(), _stream(x.device)),
           "rbffd_weights3_batch")
    return w, st


def rbffd_weights_backward(x, y, nbr, grad_w, save, status=None, m=None, n=None, order=None,
                           n_for_order=DEFAULT_N_FOR_ORDER):
    """dL/dx, dL/dy [N] from dL/dw, reusing the factors saved by rbffd_weights."""
    lib = _load()
    x, y, nbr, N, ks = _nodes2(x, y, nbr)
    grad_w = _dev(grad_w, torch.float64, "grad_w")
    if tuple(grad_w.shape) != (N, ks):
        raise ValueError(f"grad_w must have the shape of nbr {(N, ks)}, got {tuple(grad_w.shape)}")
    o, m_, n_, nfo, kmax = _order_args(order, m, n, n_for_order, N)
    save = _dev(save, torch.uint8, "save")
    need = _size(lib.rbffd_weights_save_size, N, kmax)
    if save.numel() < need:
        raise ValueError(f"save has {save.numel()} bytes, the factors need {need}")
    gx = torch.empty(N, dtype=torch.float64, device=x.device)
    gy = torch.empty(N, dtype=torch.float64, device=x.device)
    ws = _workspace(_size(lib.rbffd_weights_backward_workspace_size, N, ks), x.device)
    st = None if status is None else _vec(status, N, torch.int32, "status")
    _check(lib.rbffd_weights_backward(_p(x), _p(y), N, _p(nbr), ks, _p(o), m_, n_, nfo,
                                      _p(grad_w), _p(save), save.numel(), _p(st), _p(gx), _p(gy),
                                      _p(ws), ws.numel(), _stream(x.device)),
           "rbffd_weights_backward")
    return gx, gy


def rbffd_assemble_csr(nbr, w, n=None, order=None, n_for_order=DEFAULT_N_FOR_ORDER,
                       is_boundary=None):
    """CSR operator: (row_ptr int64 [N+1], col int32 [cap], val f64 [cap]).

    col/val have capacity N * max n; the first row_ptr[N] entries are valid.
    """
    lib = _load()
    nbr = _supports(nbr)
    N, ks = nbr.shape
    w = _dev(w, torch.float64, "w")
    if tuple(w.shape) != (N, ks):
        raise ValueError(f"w must have the shape of nbr {(N, ks)}, got {tuple(w.shape)}")
    if order is None:
        if n is None:
            raise ValueError("give n or a per-node order")
        o, nfo, nmax = None, None, int(n)
    else:
        o, nfo, nmax = _vec(order, N, torch.int8, "order"), _n_for_order(n_for_order), \
            max(n_for_order)
    b = None if is_boundary is None else _vec(is_boundary, N, torch.uint8, "is_boundary")
    cap = N * nmax
    row_ptr = torch.empty(N + 1, dtype=torch.int64, device=nbr.device)
    col = torch.empty(cap, dtype=torch.int32, device=nbr.device)
    val = torch.empty(cap, dtype=torch.float64, device=nbr.device)
    ws = _workspace(_size(lib.rbffd_assemble_csr_workspace_size, N), nbr.device)
    _check(lib.rbffd_assemble_csr(N, _p(nbr), ks, _p(o), -1 if n is None else int(n), nfo,
                                  _p(w), _p(b), _p(row_ptr), _p(col), _p(val), cap, _p(ws),
                                  ws.numel(), _stream(nbr.device)), "rbffd_assemble_csr")
    return row_ptr, col, val


def rbffd_spmv(row_ptr, col, val, u, f=None, out=None):
    """y = W u - f (f optional) for a CSR matrix."""
    lib = _load()
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    n = row_ptr.numel() - 1
    if n < 1:
        raise ValueError("row_ptr must have at least two entries")
    if col.numel() != val.numel():
        raise ValueError(f"col ({col.numel()}) and val ({val.numel()}) differ in length")
    # the operator is square (one column per node): u has one entry per row
    u = _vec(u, n, torch.float64, "u")
    fz = None if f is None else _vec(f, n, torch.float64, "f")
    y = _out(out, (n,), torch.float64, "out", u.device)
    _check(lib.rbffd_spmv(n, _p(row_ptr), _p(col), _p(val), _p(u), _p(fz), _p(y),
                          _stream(u.device)), "rbffd_spmv")
    return y


def rbffd_solve(row_ptr, col, val, b, x0=None, rtol: float = 1e-10, max_iter: int = 20000):
    """Solve W x = b (CSR W, BiCGSTAB on the GPU).  Returns (x, iterations,
    relative true residual ||b - W x|| / ||b||, info = SOLVE_*).  Synchronizes
    the stream."""
    lib = _load()
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    n = row_ptr.numel() - 1
    if col.numel() != val.numel():
        raise ValueError(f"col ({col.numel()}) and val ({val.numel()}) differ in length")
    b = _vec(b, n, torch.float64, "b")
    x = torch.zeros_like(b) if x0 is None else _vec(x0, n, torch.float64, "x0").clone()
    ws = _workspace(_size(lib.rbffd_solve_workspace_size, n), b.device)
    it, rr, info = ctypes.c_int32(0), ctypes.c_double(0.0), ctypes.c_int32(0)
    _check(lib.rbffd_solve(n, _p(row_ptr), _p(col), _p(val), _p(b), _p(x), float(rtol),
                           int(max_iter), ctypes.byref(it), ctypes.byref(rr), ctypes.byref(info),
                           _p(ws), ws.numel(), _stream(b.device)), "rbffd_solve")
    return x, it.value, rr.value, info.value


PRECOND_NONE, PRECOND_JACOBI = 0, 1


class SolveResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("info", ctypes.c_int32), ("relres", ctypes.c_double)]


def rbffd_solve_async(row_ptr, col, val, b, x, rtol: float = 1e-10, max_iter: int = 2000,
                      precond: int = PRECOND_JACOBI, result=None, workspace=None):
    """Enqueue the solve of W x = b in place on x (the initial guess), without
    host synchronisation (capturable in a graph).  result: an int8 device
    tensor of 16 bytes receiving {iters, info, relres} (see
    solve_result()); workspace: optional, rbffd_solve_workspace_size bytes.
    Returns (x, result, workspace)."""
    lib = _load()
    row_ptr = _dev(row_ptr, torch.int64, "row_ptr")
    col = _dev(col, torch.int32, "col")
    val = _dev(val, torch.float64, "val")
    n = row_ptr.numel() - 1
    if col.numel() != val.numel():
        raise ValueError(f"col ({col.numel()}) and val ({val.numel()}) differ in length")
    b = _vec(b, n, torch.float64, "b")
    x = _out(x, (n,), torch.float64, "x", b.device)
    need = _size(lib.rbffd_solve_workspace_size, n)
    if workspace is None:
        workspace = _workspace(need, b.device)
    elif not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or \
            workspace.dtype != torch.uint8 or workspace.numel() < need or \
            not workspace.is_contiguous():
        raise ValueError(f"workspace must be a contiguous uint8 GPU tensor of >= {need} bytes")
    result = _out(result, (ctypes.sizeof(SolveResult),), torch.int8, "result", b.device)
    _check(lib.rbffd_solve_async(n, _p(row_ptr), _p(col), _p(val), _p(b), _p(x), float(rtol),
                                 int(max_iter), int(precond), _p(result), _p(workspace),
                                 workspace.numel(), _stream(b.device)), "rbffd_solve_async")
    return x, result, workspace


def solve_result(result) -> tuple:
    """(iterations, relative true residual, info) from a result tensor
    (synchronises with the device)."""
    raw = bytes(result.cpu().numpy().tobytes())
    r = SolveResult.from_buffer_copy(raw)
    return r.iters, r.relres, r.info


def rbffd_time_steps(nbr, w, n: int, f, u, dt: float, n_steps: int, is_boundary=None,
                     u_work=None, workspace=None):
    """n_steps of the explicit pseudo-time loop of eq. (3), in place on u:
    u <- u + dt (f + sum_k w u[nbr]) at interior nodes.  Returns u."""
    lib = _load()
    nbr = _supports(nbr)
    N, ks = nbr.shape
    w = _dev(w, torch.float64, "w")
    if tuple(w.shape) != (N, ks):
        raise ValueError(f"w must have the shape of nbr {(N, ks)}, got {tuple(w.shape)}")
    f = _vec(f, N, torch.float64, "f")
    u = _out(u, (N,), torch.float64, "u", f.device)
    b = None if is_boundary is None else _vec(is_boundary, N, torch.uint8, "is_boundary")
    work = _out(u_work, (N,), torch.float64, "u_work", f.device)
    ws = _workspace(_size(lib.rbffd_time_steps_workspace_size, N, max(int(n), 1)), u.device) \
        if workspace is None else _dev(workspace, torch.uint8, "workspace")
    _check(lib.rbffd_time_steps(N, _p(nbr), ks, int(n), _p(w), _p(b), _p(f), float(dt),
                                int(n_steps), _p(u), _p(work), _p(ws), ws.numel(),
                                _stream(u.device)), "rbffd_time_steps")
    return u


class _WeightsFn(torch.autograd.Function):
    """w = weights(x, y) with the adjoint kernel as backward (supports fixed)."""

    @staticmethod
    def forward(ctx, x, y, nbr, m, n, order, n_for_order):
        w, st, sv = rbffd_weights(x, y, nbr, m=m, n=n, order=order, n_for_order=n_for_order,
                                  save=True)
        ctx.save_for_backward(x, y, nbr, st, sv, order if order is not None else torch.empty(0))
        ctx.has_order = order is not None
        ctx.mn = (m, n, tuple(n_for_order))
        ctx.mark_non_differentiable(st)
        return w, st

    @staticmethod
    def backward(ctx, gw, _gst):
        x, y, nbr, st, sv, order = ctx.saved_tensors
        m, n, nfo = ctx.mn
        gx, gy = rbffd_weights_backward(x, y, nbr, gw.contiguous(), sv, status=st, m=m, n=n,
                                        order=order if ctx.has_order else None, n_for_order=nfo)
        return gx, gy, None, None, None, None, None


def weights(x, y, nbr, m=None, n=None, order=None, n_for_order=DEFAULT_N_FOR_ORDER):
    """Differentiable weights: (w, status).  When x or y requires grad, the
    forward stores its LU factors and backward runs rbffd_weights_backward."""
    if x.requires_grad or y.requires_grad:
        return _WeightsFn.apply(x, y, nbr, m, n, order, n_for_order)
    w, st, _ = rbffd_weights(x, y, nbr, m=m, n=n, order=order, n_for_order=n_for_order)
    return w, st
