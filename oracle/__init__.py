"""CPU oracle: plain, slow, obviously correct reference for the GPU path.

TEST INFRASTRUCTURE.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
library never calls it and shares no code with it: the arithmetic lives in
``oracle.c`` (compiled with gcc, no fast-math, no FMA contraction) and this
module only marshals numpy arrays into it.

Functions follow the paper's definitions:
  * COO assembly: paper Sec. 5 (A is the sum of the triplet contributions;
    negative indices ignored);
  * SpMV / SpMV^T / SpMM: y = A x, y = A^T x, Y = A X;
  * Jacobi-PCG: paper Sec. 6 (PETSc CG built from MatMult, dot, AXPY and a
    residual test), textbook Hestenes-Stiefel form;
  * mixed-precision refinement: paper Sec. 2 multiprecision plan (fp32
    device data under an fp64 solver);
  * adjoint gradient: chain rule through u = A^-1 b and the assembly sum.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {0: "ok", -1: "invalid argument", -2: "index out of range", -4: "zero diagonal",
          -5: "not converged", -6: "breakdown"}


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11", "-fopenmp", "-fPIC",
               "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_i64ref = ctypes.POINTER(ctypes.c_int64)
_dref = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        lib.oracle_coo_pattern.argtypes = [_i64, _i64, _i32p, _i32p, _i32p, _i32p, _i64p, _i32p,
                                           _i64ref, _i64ref]
        lib.oracle_coo_pattern.restype = ctypes.c_int
        lib.oracle_coo_values.argtypes = [_i64, _i64p, _i32p, _f64p, ctypes.c_int, _f64p]
        lib.oracle_coo_values.restype = None
        lib.oracle_coo_slots.argtypes = [_i64, _i64, _i64p, _i32p, _i32p]
        lib.oracle_coo_slots.restype = None
        lib.oracle_coo_rows.argtypes = [_i64, _i64, _i32p, _i32p, _f64p, _i64, _i32p, _i64p, _i32p,
                                        _f64p, _i64]
        lib.oracle_coo_rows.restype = ctypes.c_int64
        lib.oracle_spmv.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p]
        lib.oracle_spmv.restype = None
        lib.oracle_spmv_transpose.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p]
        lib.oracle_spmv_transpose.restype = None
        lib.oracle_spmm.argtypes = [_i64, _i32p, _i32p, _f64p, _i64, _f64p, _i64, _f64p, _i64]
        lib.oracle_spmm.restype = None
        lib.oracle_pcg.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_double, _i64,
                                   _i64ref, _dref]
        lib.oracle_pcg.restype = ctypes.c_int
        lib.oracle_pcg_mixed.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p, ctypes.c_double,
                                         ctypes.c_double, _i64, _i64, ctypes.c_int, _i64ref,
                                         _i64ref, _dref]
        lib.oracle_pcg_mixed.restype = ctypes.c_int
        lib.oracle_sddmm.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p]
        lib.oracle_sddmm.restype = None
        lib.oracle_coo_grad.argtypes = [_i64, _i32p, _i32p, _f64p, _f64p, _f64p]
        lib.oracle_coo_grad.restype = None
        lib.oracle_block_reduce.argtypes = [_i64, _i64, _f64p, _f64p, _f64p]
        lib.oracle_block_reduce.restype = None
        lib.oracle_pcg_single_reduction.argtypes = lib.oracle_pcg.argtypes
        lib.oracle_pcg_single_reduction.restype = ctypes.c_int
        lib.oracle_vec_coo.argtypes = [_i64, _i64, _i32p, _f64p, ctypes.c_int, _f64p]
        lib.oracle_vec_coo.restype = ctypes.c_int
        lib.oracle_bicg.argtypes = lib.oracle_pcg.argtypes
        lib.oracle_bicg.restype = ctypes.c_int
        lib.oracle_pcg_pipelined.argtypes = lib.oracle_pcg.argtypes
        lib.oracle_pcg_pipelined.restype = ctypes.c_int
        lib.oracle_tfqmr.argtypes = lib.oracle_pcg.argtypes + [_dref]
        lib.oracle_tfqmr.restype = ctypes.c_int
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = None
        lib.oracle_get_threads.argtypes = []
        lib.oracle_get_threads.restype = ctypes.c_int
        for name in ("oracle_lbfgs_recursive", "oracle_lbfgs_dense"):
            fn = getattr(lib, name)
            fn.argtypes = [_i64, _i64, _f64p, _f64p, _f64p, _f64p, _f64p]
            fn.restype = None
        _lib = lib
    return _lib


def set_threads(nthreads: int) -> None:
    """OpenMP threads of the products, vector updates and dot blocks (the
    results are bitwise the same for any count)."""
    _load().oracle_set_threads(int(nthreads))


def get_threads() -> int:
    return int(_load().oracle_get_threads())


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


@dataclass
class CsrMatrix:
    """Oracle-assembled CSR matrix plus its COO helper maps."""

    n: int
    rowptr: np.ndarray  # int32[n+1]
    col: np.ndarray  # int32[nnz]
    val: np.ndarray  # float64[nnz]
    jmap: np.ndarray  # int64[nnz+1]
    perm: np.ndarray  # int32[nvalid]
    ncoo: int

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def nvalid(self) -> int:
        return int(self.perm.shape[0])


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _cf(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def coo_pattern(n: int, i: np.ndarray, j: np.ndarray):
    """Symbolic stage: (rowptr, col, jmap, perm) of the kept triplets."""
    lib = _load()
    i = _c32(i)
    j = _c32(j)
    ncoo = int(i.shape[0])
    rowptr = np.zeros(n + 1, np.int32)
    col = np.zeros(max(ncoo, 1), np.int32)
    jmap = np.zeros(ncoo + 1, np.int64)
    perm = np.zeros(max(ncoo, 1), np.int32)
    nnz = ctypes.c_int64(0)
    nvalid = ctypes.c_int64(0)
    st = lib.oracle_coo_pattern(n, ncoo, i, j, rowptr, col, jmap, perm, ctypes.byref(nnz),
                                ctypes.byref(nvalid))
    if st != 0:
        raise OracleError(st, "coo_pattern")
    return rowptr, col[:nnz.value].copy(), jmap[:nnz.value + 1].copy(), perm[:nvalid.value].copy()


def coo_values(jmap: np.ndarray, perm: np.ndarray, v: np.ndarray, mode: int = 0,
               val: np.ndarray | None = None) -> np.ndarray:
    """Numeric stage: in-order sums (INSERT, mode 0) or added sums (ADD, 1)."""
    lib = _load()
    nnz = int(jmap.shape[0]) - 1
    out = np.zeros(max(nnz, 1), np.float64) if val is None else _cf(val).copy()
    lib.oracle_coo_values(nnz, np.ascontiguousarray(jmap, np.int64), _c32(perm) if perm.size else
                          np.zeros(1, np.int32), _cf(v) if v.size else np.zeros(1), mode, out)
    return out[:nnz]


def assemble(n: int, i: np.ndarray, j: np.ndarray, v: np.ndarray) -> CsrMatrix:
    rowptr, col, jmap, perm = coo_pattern(n, i, j)
    val = coo_values(jmap, perm, np.asarray(v, np.float64))
    return CsrMatrix(n, rowptr, col, val, jmap, perm, int(np.asarray(i).shape[0]))


def coo_slots(A: CsrMatrix) -> np.ndarray:
    lib = _load()
    kslot = np.zeros(max(A.ncoo, 1), np.int32)
    lib.oracle_coo_slots(A.ncoo, A.nnz, A.jmap, A.perm if A.perm.size else np.zeros(1, np.int32),
                         kslot)
    return kslot[:A.ncoo]


def coo_rows(n: int, i, j, v, rows, max_out: int | None = None):
    """Entries of a sorted sample of rows, computed straight from the
    triplets (no full assembly).  Returns (ptr, col, val)."""
    lib = _load()
    rows = _c32(rows)
    if max_out is None:
        max_out = 64 * len(rows) + 64
    ptr = np.zeros(len(rows) + 1, np.int64)
    col = np.zeros(max_out, np.int32)
    val = np.zeros(max_out, np.float64)
    w = lib.oracle_coo_rows(n, int(np.asarray(i).shape[0]), _c32(i), _c32(j), _cf(v), len(rows),
                            rows, ptr, col, val, max_out)
    if w < 0:
        raise OracleError(int(w), "coo_rows")
    return ptr, col[:w].copy(), val[:w].copy()


def spmv(A: CsrMatrix, x: np.ndarray) -> np.ndarray:
    lib = _load()
    y = np.empty(A.n, np.float64)
    lib.oracle_spmv(A.n, A.rowptr, A.col if A.nnz else np.zeros(1, np.int32),
                    A.val if A.nnz else np.zeros(1), _cf(x), y)
    return y


def spmv_transpose(A: CsrMatrix, x: np.ndarray) -> np.ndarray:
    lib = _load()
    y = np.empty(A.n, np.float64)
    lib.oracle_spmv_transpose(A.n, A.rowptr, A.col if A.nnz else np.zeros(1, np.int32),
                              A.val if A.nnz else np.zeros(1), _cf(x), y)
    return y


def abs_spmv(A: CsrMatrix, x: np.ndarray) -> np.ndarray:
    """|A| |x|, the scale of the componentwise SpMV error bound."""
    B = CsrMatrix(A.n, A.rowptr, A.col, np.abs(A.val), A.jmap, A.perm, A.ncoo)
    return spmv(B, np.abs(x))


def abs_spmv_transpose(A: CsrMatrix, x: np.ndarray) -> np.ndarray:
    B = CsrMatrix(A.n, A.rowptr, A.col, np.abs(A.val), A.jmap, A.perm, A.ncoo)
    return spmv_transpose(B, np.abs(x))


def spmm(A: CsrMatrix, X: np.ndarray) -> np.ndarray:
    lib = _load()
    X = _cf(X)
    nrhs = X.shape[1]
    Y = np.empty((A.n, nrhs), np.float64)
    lib.oracle_spmm(A.n, A.rowptr, A.col, A.val, nrhs, X, nrhs, Y, nrhs)
    return Y


@dataclass
class CgResult:
    x: np.ndarray
    iters: int
    relres: float
    status: int


def pcg(A: CsrMatrix, b: np.ndarray, rtol: float, maxit: int = 100000,
        x0: np.ndarray | None = None) -> CgResult:
    lib = _load()
    x = np.zeros(A.n) if x0 is None else _cf(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_pcg(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol, maxit, ctypes.byref(it),
                        ctypes.byref(rr))
    return CgResult(x, it.value, rr.value, st)


def pcg_single_reduction(A: CsrMatrix, b: np.ndarray, rtol: float, maxit: int = 100000,
                         x0: np.ndarray | None = None) -> CgResult:
    """Chronopoulos-Gear Jacobi-PCG (one reduction point per iteration)."""
    lib = _load()
    x = np.zeros(A.n) if x0 is None else _cf(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_pcg_single_reduction(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol, maxit,
                                         ctypes.byref(it), ctypes.byref(rr))
    return CgResult(x, it.value, rr.value, st)


def pcg_pipelined(A: CsrMatrix, b: np.ndarray, rtol: float, maxit: int = 100000,
                  x0: np.ndarray | None = None) -> CgResult:
    """Pipelined (Ghysels-Vanroose) Jacobi-PCG: one reduction per iteration,
    overlappable with the next product."""
    lib = _load()
    x = np.zeros(A.n) if x0 is None else _cf(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_pcg_pipelined(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol, maxit,
                                  ctypes.byref(it), ctypes.byref(rr))
    return CgResult(x, it.value, rr.value, st)


def bicg(A: CsrMatrix, b: np.ndarray, rtol: float, maxit: int = 100000,
         x0: np.ndarray | None = None) -> CgResult:
    """Jacobi-preconditioned BiCG, shadow residual started at the residual."""
    lib = _load()
    x = np.zeros(A.n) if x0 is None else _cf(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_bicg(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol, maxit, ctypes.byref(it),
                         ctypes.byref(rr))
    return CgResult(x, it.value, rr.value, st)


@dataclass
class TfqmrResult:
    x: np.ndarray
    iters: int  # half-steps, one product with A each
    relres: float
    status: int
    bound: float  # sqrt(m + 1) tau_m at exit, an upper bound of ||b - A x||


def tfqmr(A: CsrMatrix, b: np.ndarray, rtol: float, maxit: int = 100000,
          x0: np.ndarray | None = None) -> TfqmrResult:
    """Right-Jacobi-preconditioned TFQMR; stops on its residual bound."""
    lib = _load()
    x = np.zeros(A.n) if x0 is None else _cf(x0).copy()
    it = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    bd = ctypes.c_double(0.0)
    st = lib.oracle_tfqmr(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol, maxit, ctypes.byref(it),
                          ctypes.byref(rr), ctypes.byref(bd))
    return TfqmrResult(x, it.value, rr.value, st, bd.value)


def _lbfgs(fn, S, Y, g, h0):
    S = np.asfortranarray(S, np.float64)  # column j contiguous
    Y = np.asfortranarray(Y, np.float64)
    n, m = S.shape
    p = np.empty(n)
    fn(n, m, S.ravel(order="F"), Y.ravel(order="F"), _cf(g), _cf(h0), p)
    return p


def lbfgs_recursive(S, Y, g, h0):
    """p = H g by the two-loop recursion; S, Y: n x m, oldest pair first."""
    return _lbfgs(_load().oracle_lbfgs_recursive, S, Y, g, h0)


def lbfgs_dense(S, Y, g, h0):
    """p = H g by the intermediate dense formula (triangular solves with
    R = triu(S^T Y))."""
    return _lbfgs(_load().oracle_lbfgs_dense, S, Y, g, h0)


@dataclass
class MixedResult:
    x: np.ndarray
    outer: int
    inner: int
    relres: float
    status: int


def pcg_mixed(A: CsrMatrix, b: np.ndarray, rtol_outer: float = 1e-10, rtol_inner: float = 1e-4,
              maxit_outer: int = 100, maxit_inner: int = 100000,
              early_exit: bool = False) -> MixedResult:
    """FP32-inner / FP64-outer refinement.  The inner solve stops at
    rtol_inner relative to its right-hand side; with ``early_exit`` also as
    soon as its residual is below rtol_outer ||b|| / 2."""
    lib = _load()
    x = np.zeros(A.n)
    outer = ctypes.c_int64(0)
    inner = ctypes.c_int64(0)
    rr = ctypes.c_double(0.0)
    st = lib.oracle_pcg_mixed(A.n, A.rowptr, A.col, A.val, _cf(b), x, rtol_outer, rtol_inner,
                              maxit_outer, maxit_inner, 1 if early_exit else 0,
                              ctypes.byref(outer), ctypes.byref(inner), ctypes.byref(rr))
    return MixedResult(x, outer.value, inner.value, rr.value, st)


def sddmm(A: CsrMatrix, lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    lib = _load()
    G = np.empty(max(A.nnz, 1), np.float64)
    lib.oracle_sddmm(A.n, A.rowptr, A.col, _cf(lam), _cf(u), G)
    return G[:A.nnz]


def coo_grad(i, j, lam, u) -> np.ndarray:
    lib = _load()
    i = _c32(i)
    gv = np.empty(max(i.shape[0], 1), np.float64)
    lib.oracle_coo_grad(i.shape[0], i, _c32(j), _cf(lam), _cf(u), gv)
    return gv[:i.shape[0]]


def block_reduce(grad_v: np.ndarray, dv: np.ndarray, block: int) -> np.ndarray:
    lib = _load()
    nb = grad_v.shape[0] // block
    out = np.empty(nb, np.float64)
    lib.oracle_block_reduce(nb, block, _cf(grad_v), _cf(dv), out)
    return out


def vec_coo(n: int, i, v, x, mode: int = 0) -> np.ndarray:
    """COO vector assembly into a copy of x (paper Sec. 5, VecSetValuesCOO)."""
    lib = _load()
    i = _c32(i)
    out = _cf(x).copy()
    st = lib.oracle_vec_coo(n, i.shape[0], i if i.size else np.zeros(1, np.int32),
                            _cf(v) if i.size else np.zeros(1), mode, out)
    if st != 0:
        raise OracleError(st, "vec_coo")
    return out
