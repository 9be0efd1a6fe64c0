"""CPU oracle for the RBF-FD Laplacian stencil-weight path (FP64).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package.  It shares no code with the HIP library.

The arithmetic lives in ``rbffd_oracle.c`` (plain C, one stencil at a time);
this module builds it with gcc and wraps it with ctypes.  Each wrapper names
the part of the paper it follows; see the C file's header for the exact
definitions (orderings, rounding, status codes).

Pins (tests/test_oracle_*.py) tie every function to something other than
itself: brute-force and k-d tree kNN, polynomial reproduction, the classical
five-point Laplacian, scale/rigid-motion invariance, lattice symmetry,
LAPACK and exact rational solves, the convergence order of the Poisson
solution, central finite differences of the adjoint, and SciPy's CSR
product.  ``solve`` (the assembled system's solution) is SciPy's direct
solver itself, pinned by its residual and by the convergence order.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rbffd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

# Status codes of the specification (same values as the library's).
OK, SINGULAR, FELL_BACK, NONFINITE, BAD_INDEX, DUPLICATE = 0, 1, 2, 3, 4, 5


def build(force: bool = True) -> str:
    """Compile the oracle into liboracle.so with gcc (no FMA contraction)."""
    if not force and os.path.exists(_LIB) and \
            os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            build(force=False)
            lib = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            I64 = ctypes.c_int64
            I32 = ctypes.c_int32
            lib.oracle_knn.argtypes = [I64, P, P, I32, P, I64, P]
            lib.oracle_assemble.argtypes = [I64, P, P, I64, P, ctypes.c_int,
                                            ctypes.c_int, P, P, P]
            lib.oracle_lu.argtypes = [ctypes.c_int, P, P, P]
            lib.oracle_lu32.argtypes = [ctypes.c_int, P, P, P]
            lib.oracle_lu_solve.argtypes = [ctypes.c_int, P, P, P, P]
            lib.oracle_lu_solve.restype = None
            lib.oracle_weights.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                           P, I64, P, P]
            lib.oracle_weights_op.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                              P, I64, I32, P, P]
            lib.oracle_weights_mixed.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                                 P, I64, P, P, P]
            lib.oracle_weights_mixed_form.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                                      P, I64, P, P, P, I32]
            lib.oracle_weights_mixed_op.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                                    P, I64, P, P, P, I32, I32]
            lib.oracle_gj32.argtypes = [ctypes.c_int, P, P]
            lib.oracle_adjoint.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                           P, P, P]
            lib.oracle_adjoint_rows.argtypes = [I64, P, P, P, I32, P, I32, I32, P,
                                                P, P, I64, P, P]
            lib.oracle_csr.argtypes = [I64, P, I32, P, I32, P, P, P, P, P, P]
            lib.oracle_spmv.argtypes = [I64, P, P, P, P, P, P]
            lib.oracle_knn3.argtypes = [I64, P, P, P, I32, P, I64, P]
            lib.oracle_assemble3.argtypes = [I64, P, P, P, I64, P, ctypes.c_int,
                                             ctypes.c_int, P, P, P]
            lib.oracle_weights3.argtypes = [I64, P, P, P, P, I32, I32, I32, P, I64, P, P]
            lib.oracle_weights3_op.argtypes = [I64, P, P, P, P, I32, I32, I32, P, I64, I32,
                                               P, P]
            lib.oracle_time_steps.argtypes = [I64, P, I32, I32, P, P, P, ctypes.c_double,
                                              I64, P]
            _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _check_supports(x, y, nbr, k_stride=None):
    """The C routines index nbr as [len(x)][k_stride]: refuse other shapes."""
    if y.shape != x.shape or nbr.ndim != 2 or nbr.shape[0] != x.shape[0]:
        raise ValueError(f"need x, y [N] and nbr [N, k]; got {x.shape}, {y.shape}, {nbr.shape}")
    if k_stride is not None and k_stride != nbr.shape[1]:
        raise ValueError(f"k_stride {k_stride} != nbr.shape[1] {nbr.shape[1]}")


def n_monomials(m: int) -> int:
    return (m + 1) * (m + 2) // 2


def knn(x, y, k: int, queries=None) -> np.ndarray:
    """Support selection N(x) of eq. (1): the k nearest nodes, ascending by
    (d^2, index), brute force.  Returns int32 [len(queries) or N, k]."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = x.shape[0] if q is None else q.shape[0]
    out = np.empty((nq, k), dtype=np.int32)
    rc = lib.oracle_knn(x.shape[0], _p(x), _p(y), k, _p(q), nq, _p(out))
    if rc != 0:
        raise ValueError(f"oracle_knn: error {rc}")
    return out


def n_monomials3(m: int) -> int:
    return (m + 1) * (m + 2) * (m + 3) // 6


def knn3(x, y, z, k: int, queries=None) -> np.ndarray:
    """N(x) of eq. (1) for nodes in R^3: the k nearest nodes, ascending by
    (d^2, index), brute force.  Returns int32 [len(queries) or N, k]."""
    lib = _load()
    x, y, z = _f64(x), _f64(y), _f64(z)
    q = None if queries is None else np.ascontiguousarray(queries, dtype=np.int64)
    nq = x.shape[0] if q is None else q.shape[0]
    out = np.empty((nq, k), dtype=np.int32)
    rc = lib.oracle_knn3(x.shape[0], _p(x), _p(y), _p(z), k, _p(q), nq, _p(out))
    if rc != 0:
        raise ValueError(f"oracle_knn3: error {rc}")
    return out


def assemble3(x, y, z, i: int, idx, m: int):
    """The 3-D augmented system of node i on support idx (r^3, monomials of
    degree <= m in x, y, z).  Returns (status, M [K,K], rhs [K], s)."""
    lib = _load()
    x, y, z, idx = _f64(x), _f64(y), _f64(z), _i32(idx)
    n = idx.shape[0]
    K = n + n_monomials3(m)
    M = np.zeros((K, K))
    rhs = np.zeros(K)
    s = np.zeros(1)
    st = lib.oracle_assemble3(x.shape[0], _p(x), _p(y), _p(z), i, _p(idx), n, m,
                              _p(M), _p(rhs), _p(s))
    return st, M, rhs, float(s[0])


def weights3(x, y, z, nbr, m: int, n: int, rows=None):
    """Laplacian weights of eq. (1) in three dimensions, uniform (m, n).
    Returns (w [rows, k_stride], status [rows])."""
    lib = _load()
    x, y, z, nbr = _f64(x), _f64(y), _f64(z), _i32(nbr)
    if nbr.ndim != 2 or nbr.shape[0] != x.shape[0] or y.shape != x.shape or z.shape != x.shape:
        raise ValueError("x, y, z must be [N] and nbr [N, k_stride]")
    N, ks = x.shape[0], nbr.shape[1]
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    w = np.empty((nr, ks))
    st = np.empty(nr, dtype=np.int32)
    rc = lib.oracle_weights3(N, _p(x), _p(y), _p(z), _p(nbr), ks, m, n, _p(r), nr,
                             _p(w), _p(st))
    if rc != 0:
        raise ValueError(f"oracle_weights3: error {rc}")
    return w, st


D3_DX, D3_DY, D3_DZ = 1, 2, 3


def weights3_op(x, y, z, nbr, m: int, n: int, op: int, rows=None):
    """Weights of eq. (1) in three dimensions for op (0 Laplacian, D3_DX,
    D3_DY, D3_DZ), uniform (m, n).  Returns (w [rows, k_stride], status)."""
    lib = _load()
    x, y, z, nbr = _f64(x), _f64(y), _f64(z), _i32(nbr)
    if nbr.ndim != 2 or nbr.shape[0] != x.shape[0] or y.shape != x.shape or z.shape != x.shape:
        raise ValueError("x, y, z must be [N] and nbr [N, k_stride]")
    N, ks = x.shape[0], nbr.shape[1]
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    w = np.empty((nr, ks))
    st = np.empty(nr, dtype=np.int32)
    rc = lib.oracle_weights3_op(N, _p(x), _p(y), _p(z), _p(nbr), ks, m, n, _p(r), nr, int(op),
                                _p(w), _p(st))
    if rc != 0:
        raise ValueError(f"oracle_weights3_op: error {rc}")
    return w, st


def assemble(x, y, i: int, idx, m: int):
    """The augmented PHS + monomial system of node i on support idx.
    Returns (status, M [K,K], rhs [K], s)."""
    lib = _load()
    x, y, idx = _f64(x), _f64(y), _i32(idx)
    n = idx.shape[0]
    K = n + n_monomials(m)
    M = np.zeros((K, K))
    rhs = np.zeros(K)
    s = np.zeros(1)
    st = lib.oracle_assemble(x.shape[0], _p(x), _p(y), i, _p(idx), n, m,
                             _p(M), _p(rhs), _p(s))
    return st, M, rhs, float(s[0])


def lu(M):
    """Partial-pivoting LU (in a copy).  Returns (status, LU, perm, dinv)."""
    lib = _load()
    A = _f64(M).copy()
    K = A.shape[0]
    perm = np.zeros(K, dtype=np.int32)
    dinv = np.zeros(K)
    st = lib.oracle_lu(K, _p(A), _p(perm), _p(dinv))
    return st, A, perm, dinv


def lu32(M):
    """The FP32 factorisation of the mixed form (in a float32 copy of M).
    Returns (status, LU, perm, dinv) as ``lu``, in float32."""
    lib = _load()
    A = np.ascontiguousarray(M, dtype=np.float32).copy()
    K = A.shape[0]
    perm = np.zeros(K, dtype=np.int32)
    dinv = np.zeros(K, dtype=np.float32)
    st = lib.oracle_lu32(K, _p(A), _p(perm), _p(dinv))
    return st, A, perm, dinv


def gj32(M):
    """The FP32 Gauss-Jordan inversion of the mixed form's second reading (in
    a float32 copy of M).  Returns (status, S, perm): S = (P M)^-1 in
    float32, P the row swaps perm[c] <-> c taken in column order."""
    lib = _load()
    A = np.ascontiguousarray(M, dtype=np.float32).copy()
    K = A.shape[0]
    perm = np.zeros(K, dtype=np.int32)
    st = lib.oracle_gj32(K, _p(A), _p(perm))
    return st, A, perm


def lu_solve(LU, perm, dinv, b):
    lib = _load()
    LU = _f64(LU)
    out = _f64(b).copy()
    lib.oracle_lu_solve(LU.shape[0], _p(LU), _p(_i32(perm)), _p(_f64(dinv)), _p(out))
    return out


def weights(x, y, nbr, m: int | None = None, n: int | None = None, order=None,
            n_for_m=(12, 30, 56), rows=None, k_stride: int | None = None):
    """Weights of eq. (1) for the Laplacian.  Uniform (m, n) or per-node order.
    Returns (w [rows, k_stride], status [rows])."""
    lib = _load()
    x, y, nbr = _f64(x), _f64(y), _i32(nbr)
    _check_supports(x, y, nbr, k_stride)
    N = x.shape[0]
    ks = nbr.shape[1] if k_stride is None else k_stride
    nfm = _i32(n_for_m)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int8)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    w = np.empty((nr, ks))
    st = np.empty(nr, dtype=np.int32)
    rc = lib.oracle_weights(N, _p(x), _p(y), _p(nbr), ks, _p(o),
                            -1 if m is None else m, -1 if n is None else n,
                            _p(nfm), _p(r), nr, _p(w), _p(st))
    if rc != 0:
        raise ValueError(f"oracle_weights: error {rc}")
    return w, st


LAPLACIAN, D_DX, D_DY = 0, 1, 2


def weights_op(x, y, nbr, m: int, n: int, op: int, rows=None):
    """Weights of eq. (1) for the operator op (LAPLACIAN, D_DX, D_DY: the
    right-hand side [L phi_k; L p_j] of that operator at the centre), uniform
    (m, n).  Returns (w [rows, k], status [rows])."""
    lib = _load()
    x, y, nbr = _f64(x), _f64(y), _i32(nbr)
    _check_supports(x, y, nbr)
    N, ks = x.shape[0], nbr.shape[1]
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    w = np.empty((nr, ks))
    st = np.empty(nr, dtype=np.int32)
    rc = lib.oracle_weights_op(N, _p(x), _p(y), _p(nbr), ks, None, m, n, None, _p(r), nr,
                               int(op), _p(w), _p(st))
    if rc != 0:
        raise ValueError(f"oracle_weights_op: error {rc}")
    return w, st


MIXED_LU, MIXED_GJ = 0, 1


def weights_mixed(x, y, nbr, m: int | None = None, n: int | None = None, order=None,
                  n_for_m=(12, 30, 56), rows=None, k_stride: int | None = None,
                  form: int = MIXED_LU, op: int = LAPLACIAN):
    """Mixed-precision weights: FP32 factorisation of the FP64-assembled
    system + FP64 refinement, FP64 fallback.  form MIXED_LU: LU factors and
    triangular solves; MIXED_GJ: the Gauss-Jordan inverse applied as a
    product.  op: LAPLACIAN, D_DX or D_DY (the right-hand side and scale of
    weights_op).  Returns (w, status, corrections); for a stencil that fell
    back, the corrections tried before it did."""
    lib = _load()
    x, y, nbr = _f64(x), _f64(y), _i32(nbr)
    _check_supports(x, y, nbr, k_stride)
    N = x.shape[0]
    ks = nbr.shape[1] if k_stride is None else k_stride
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int8)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    nr = N if r is None else r.shape[0]
    w = np.empty((nr, ks))
    st = np.empty(nr, dtype=np.int32)
    it = np.empty(nr, dtype=np.int32)
    rc = lib.oracle_weights_mixed_op(N, _p(x), _p(y), _p(nbr), ks, _p(o),
                                     -1 if m is None else m, -1 if n is None else n,
                                     _p(_i32(n_for_m)), _p(r), nr, _p(w), _p(st), _p(it),
                                     int(form), int(op))
    if rc != 0:
        raise ValueError(f"oracle_weights_mixed: error {rc}")
    return w, st, it


def adjoint(x, y, nbr, G, m: int | None = None, n: int | None = None, order=None,
            n_for_m=(12, 30, 56), rows=None):
    """dL/dx, dL/dy of all nodes given G = dL/dw (reverse mode of weights).
    With rows, only the listed nodes' stencils contribute (in list order)."""
    lib = _load()
    x, y, nbr, G = _f64(x), _f64(y), _i32(nbr), _f64(G)
    _check_supports(x, y, nbr)
    if G.shape != nbr.shape:
        raise ValueError(f"G {G.shape} must have the shape of nbr {nbr.shape}")
    N = x.shape[0]
    gx = np.empty(N)
    gy = np.empty(N)
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int8)
    r = None if rows is None else np.ascontiguousarray(rows, dtype=np.int64)
    rc = lib.oracle_adjoint_rows(N, _p(x), _p(y), _p(nbr), nbr.shape[1], _p(o),
                                 -1 if m is None else m, -1 if n is None else n,
                                 _p(_i32(n_for_m)), _p(G), _p(r), N if r is None else r.shape[0],
                                 _p(gx), _p(gy))
    if rc < 0:
        raise ValueError(f"oracle_adjoint: error {rc}")
    return gx, gy, rc


def csr(nbr, w, n: int | None = None, is_boundary=None, order=None,
        n_for_m=(12, 30, 56)):
    """The operator of eq. (1) as CSR; Dirichlet rows are identity rows."""
    lib = _load()
    nbr, w = _i32(nbr), _f64(w)
    N, ks = nbr.shape
    o = None if order is None else np.ascontiguousarray(order, dtype=np.int8)
    b = None if is_boundary is None else np.ascontiguousarray(is_boundary, dtype=np.uint8)
    cap = N * ks
    row_ptr = np.empty(N + 1, dtype=np.int64)
    col = np.empty(cap, dtype=np.int32)
    val = np.empty(cap)
    lib.oracle_csr(N, _p(nbr), ks, _p(o), -1 if n is None else n,
                   _p(_i32(n_for_m)), _p(w), _p(b), _p(row_ptr), _p(col), _p(val))
    nnz = int(row_ptr[-1])
    return row_ptr, col[:nnz].copy(), val[:nnz].copy()


def spmv(row_ptr, col, val, u, f=None):
    """y = W u - f, sequential fma row sums in CSR order."""
    lib = _load()
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    col, val, u = _i32(col), _f64(val), _f64(u)
    fz = None if f is None else _f64(f)
    n = row_ptr.shape[0] - 1
    y = np.empty(n)
    lib.oracle_spmv(n, _p(row_ptr), _p(col), _p(val), _p(u), _p(fz), _p(y))
    return y


def solve(row_ptr, col, val, b):
    """The solution of the assembled system W x = b (the steady Dirichlet
    problem of eq. (2) with the boundary rows of section IV), by its plain
    definition: a direct sparse LU solve (SciPy's SuperLU).  Any iterative
    method the GPU runs approximates this vector."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spl
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    n = row_ptr.shape[0] - 1
    A = sp.csc_matrix(sp.csr_matrix((_f64(val), _i32(col), row_ptr), shape=(n, n)))
    return spl.spsolve(A, _f64(b))


def time_steps(nbr, w, n: int, f, u0, dt: float, n_steps: int, is_boundary=None):
    """n_steps of the explicit loop of eq. (3); returns the final u (copy)."""
    lib = _load()
    nbr, w, f = _i32(nbr), _f64(w), _f64(f)
    N, ks = nbr.shape
    u = _f64(u0).copy()
    b = None if is_boundary is None else np.ascontiguousarray(is_boundary, dtype=np.uint8)
    rc = lib.oracle_time_steps(N, _p(nbr), ks, int(n), _p(w), _p(b), _p(f), float(dt),
                               int(n_steps), _p(u))
    if rc != 0:
        raise ValueError(f"oracle_time_steps: error {rc}")
    return u
