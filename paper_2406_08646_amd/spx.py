"""Python binding of the ``libspx`` C ABI (argument marshalling only).

Every method forwards to the ``extern "C"`` entry point of the same name in
``include/spx.h``; all arithmetic runs in the HIP kernels of ``libspx.so``.
torch supplies device memory and the current HIP stream.  If the library is
missing the binding raises instead of computing anything elsewhere.

    A = coo_preallocate(n, i, j)          # i, j: cuda int32 tensors
    A.set_values_coo(v)                   # v: cuda float64, same length
    y = A.matmult(x); yt = A.matmult_transpose(x)
    res = A.cg_solve(b, rtol=1e-10)       # res.x, res.iters, res.relres
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch  # noqa: F401  (must be loaded before libspx so both share one HIP runtime)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libspx.so")

OK = 0
INVALID_ARG = -1
INDEX_OUT_OF_RANGE = -2
HIP_ERROR = -3
ZERO_DIAGONAL = -4
NOT_CONVERGED = -5
BREAKDOWN = -6
NOT_IMPLEMENTED = -7
OUT_OF_MEMORY = -8
STATUS_NAMES = {0: "OK", -1: "INVALID_ARG", -2: "INDEX_OUT_OF_RANGE", -3: "HIP_ERROR",
                -4: "ZERO_DIAGONAL", -5: "NOT_CONVERGED", -6: "BREAKDOWN",
                -7: "NOT_IMPLEMENTED", -8: "OUT_OF_MEMORY"}
INSERT_VALUES = 0
ADD_VALUES = 1
OPT_SPMV_LANES = 1
OPT_XCD_REMAP = 2
OPT_PROFILE = 3
OPT_SPMV_VARIANT = 4
OPT_ROWS_PER_BLOCK = 5
OPT_NONTEMPORAL = 6
OPT_SOLVER_BLOCKS = 7
OPT_QUAD_LOADS = 8
OPT_VECTOR_BLOCKS = 9
OPT_PIPELINE = 10
OPT_ROWS_PER_BLOCK_F32 = 11
OPT_CG_VARIANT = 12
OPT_GRAPH = 13
OPT_SMALL_SOLVE = 14
OPT_IR_EARLY_EXIT = 15
OPT_SPMM_TILE_ROWS = 16
NOALLOC_MAX_ROWS = 2097152  # SPX_NOALLOC_MAX_ROWS
PROFILE_KINDS = ("spmv_dot_f64", "update_f64", "pupdate_f64", "spmv_dot_f32", "update_f32",
                 "pupdate_f32")

# hard failures raise; solver outcomes are returned as a status
_SOLVER_OUTCOMES = (OK, NOT_CONVERGED, BREAKDOWN, ZERO_DIAGONAL)

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_d = ctypes.c_double
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pd = ctypes.POINTER(ctypes.c_double)

_SIGNATURES = {
    "spx_coo_preallocate": [_i64, _i64, _vp, _vp, _vp, ctypes.POINTER(_vp)],
    "spx_set_values_coo": [_vp, _vp, ctypes.c_int, _vp],
    "spx_destroy": [_vp],
    "spx_matmult": [_vp, _vp, _vp, _vp],
    "spx_matmult_transpose": [_vp, _vp, _vp, _vp],
    "spx_spmm": [_vp, _i64, _vp, _i64, _vp, _i64, _vp],
    "spx_cg_solve": [_vp, _vp, _vp, _d, _i64, _i32, _vp, _pi64, _pd],
    "spx_cg_solve_noalloc": [_vp, _vp, _vp, _d, _i64, _i32, _vp, _pi64, _pd],
    "spx_cg_solve_transpose": [_vp, _vp, _vp, _d, _i64, _i32, _vp, _pi64, _pd],
    "spx_cg_solve_mixed": [_vp, _vp, _vp, _d, _d, _i64, _i64, _i32, _vp, _pi64, _pi64, _pd],
    "spx_batch_create": [_i32, ctypes.POINTER(_vp), _vp, ctypes.POINTER(_vp)],
    "spx_batch_destroy": [_vp],
    "spx_batch_total_rows": [_vp, _pi64],
    "spx_lbfgs_create": [_i64, _i32, _vp, ctypes.POINTER(_vp)],
    "spx_lbfgs_destroy": [_vp],
    "spx_lbfgs_reset": [_vp],
    "spx_lbfgs_get_info": [_vp, _pi64, ctypes.POINTER(_i32), ctypes.POINTER(_i32)],
    "spx_lbfgs_update": [_vp, _vp, _vp, _vp],
    "spx_lbfgs_apply": [_vp, _vp, _vp, _vp, _vp],
    "spx_lbfgs_update_apply": [_vp, _vp, _vp, _vp, _vp, _vp, _vp],
    "spx_set_allocator": [_vp, _vp, _vp],
    "spx_stream_copy": [_vp, _vp, _i64, _vp],
    "spx_stream_sum": [_vp, _i64, _vp, _vp],
    "spx_batch_cg": [_vp, _vp, _vp, _d, _i64, _vp, _vp, _pi64, _pd],
    "spx_batch_bicg": [_vp, _vp, _vp, _d, _i64, _vp, _vp, _pi64, _pd],
    "spx_batch_tfqmr": [_vp, _vp, _vp, _d, _i64, _vp, _vp, _pi64, _pd],
    "spx_sddmm": [_vp, _vp, _vp, _vp, _vp],
    "spx_coo_gather": [_vp, _vp, _vp, _vp],
    "spx_coo_gather_blocks": [_vp, _vp, _vp, _i64, _vp, _vp],
    "spx_get_info": [_vp, _pi64, _pi64, _pi64, _pi64],
    "spx_get_csr": [_vp, _i32, _vp, _vp, _vp, _vp],
    "spx_get_window": [_vp, _i32, _pi64, _vp, _vp, _vp, _vp],
    "spx_get_coo_maps": [_vp, _vp, _vp, _vp],
    "spx_set_option": [_vp, _i32, _i64],
    "spx_get_option": [_vp, _i32, _pi64],
    "spx_get_profile": [_vp, _i32, _pd, _pi64],
    "spx_reset_profile": [_vp],
    "spx_vec_coo_preallocate": [_i64, _i64, _vp, _vp, ctypes.POINTER(_vp)],
    "spx_vec_set_values_coo": [_vp, _vp, ctypes.c_int, _vp, _vp],
    "spx_vec_coo_get_info": [_vp, _pi64, _pi64, _pi64, _pi64],
    "spx_vec_coo_destroy": [_vp],
    "spx_split_preallocate": [_i64, _i64, _i64, _i64, _vp, _vp, _vp, ctypes.POINTER(_vp)],
    "spx_split_set_values_coo": [_vp, _vp, ctypes.c_int, _vp],
    "spx_split_matmult": [_vp, _vp, _vp, _vp, _vp],
    "spx_split_gather_ghosts": [_vp, _vp, _vp, _vp],
    "spx_split_get_info": [_vp, _pi64, _pi64, _pi64, _pi64],
    "spx_split_blocks": [_vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "spx_split_get_maps": [_vp, _vp, _vp, _vp],
    "spx_split_destroy": [_vp],
    "spx_last_error": [],
    "spx_version": [],
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libspx.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2406_08646_amd.build`")
        lib = ctypes.CDLL(path)
        for name, args in _SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = ctypes.c_char_p if name in ("spx_last_error", "spx_version") else ctypes.c_int
        _lib = lib
    return _lib


class SpxError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")
        self.code = code


def _check(rc: int, allowed=(OK,)) -> int:
    if rc not in allowed:
        msg = load_library().spx_last_error().decode(errors="replace")
        raise SpxError(rc, msg)
    return rc


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, length: Optional[int], name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if length is not None and t.numel() != length:
        raise ValueError(f"{name} must have {length} elements, got {t.numel()}")
    return t


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None or t.numel() == 0 else t.data_ptr())


@dataclass
class SolveResult:
    x: torch.Tensor
    iters: int
    relres: float
    status: int


@dataclass
class MixedResult:
    x: torch.Tensor
    outer: int
    inner: int
    relres: float
    status: int


class Matrix:
    """A matrix assembled from COO triplets on the GPU (owns a spx handle,
    or borrows one that ``owner`` keeps alive)."""

    def __init__(self, handle: ctypes.c_void_p, n: int, ncoo: int, device: torch.device,
                 owner=None):
        self._h = handle
        self.n = n
        self.ncoo = ncoo
        self.device = device
        self._owner = owner

    # -- lifetime
    def destroy(self) -> None:
        if self._h:
            if self._owner is None:
                _check(load_library().spx_destroy(self._h))
            self._h = None
            self._owner = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise RuntimeError("matrix has been destroyed")
        return self._h

    # -- assembly
    def set_values_coo(self, v: torch.Tensor, mode: int = INSERT_VALUES, stream=None) -> None:
        _dev(v, torch.float64, self.ncoo, "v")
        _check(load_library().spx_set_values_coo(self.handle, _ptr(v), mode, _stream(stream)))

    def get_info(self):
        n, nnz, nvalid, ncoo = (ctypes.c_int64() for _ in range(4))
        _check(load_library().spx_get_info(self.handle, ctypes.byref(n), ctypes.byref(nnz),
                                           ctypes.byref(nvalid), ctypes.byref(ncoo)))
        return {"n": n.value, "nnz": nnz.value, "nvalid": nvalid.value, "ncoo": ncoo.value}

    @property
    def nnz(self) -> int:
        return self.get_info()["nnz"]

    def get_csr(self, transpose: bool = False, stream=None):
        info = self.get_info()
        rowptr = torch.empty(self.n + 1, dtype=torch.int32, device=self.device)
        col = torch.empty(info["nnz"], dtype=torch.int32, device=self.device)
        val = torch.empty(info["nnz"], dtype=torch.float64, device=self.device)
        _check(load_library().spx_get_csr(self.handle, int(transpose), _ptr(rowptr), _ptr(col),
                                          _ptr(val), _stream(stream)))
        return rowptr, col, val

    def get_window(self, transpose: bool = False, arrays: bool = True, stream=None):
        """The window index (see spx_get_window): a dict with the statistics
        and, when the index exists and ``arrays``, its device arrays."""
        stats = (ctypes.c_int64 * 4)()
        lib = load_library()
        _check(lib.spx_get_window(self.handle, int(transpose), ctypes.cast(stats, _pi64), None,
                                  None, None, _stream(stream)))
        out = {"built": bool(stats[0]), "max_blocks": stats[1], "total_blocks": stats[2],
               "gather_entries": stats[3]}
        if stats[0] and arrays:
            tiles = (self.n + 255) // 256
            ptr = torch.empty(tiles + 1, dtype=torch.int32, device=self.device)
            blk = torch.empty(max(stats[2], 1), dtype=torch.int32, device=self.device)
            lcol = torch.empty(self.nnz, dtype=torch.uint16, device=self.device)
            _check(lib.spx_get_window(self.handle, int(transpose), ctypes.cast(stats, _pi64),
                                      _ptr(ptr), _ptr(blk), _ptr(lcol), _stream(stream)))
            out.update(ptr=ptr, blk=blk[:stats[2]], lcol=lcol)
        return out

    def get_coo_maps(self, stream=None):
        info = self.get_info()
        jmap = torch.empty(info["nnz"] + 1, dtype=torch.int32, device=self.device)
        perm = torch.empty(info["nvalid"], dtype=torch.int32, device=self.device)
        _check(load_library().spx_get_coo_maps(self.handle, _ptr(jmap), _ptr(perm),
                                               _stream(stream)))
        return jmap, perm

    # -- products
    def matmult(self, x: torch.Tensor, y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        _dev(x, torch.float64, self.n, "x")
        y = torch.empty_like(x) if y is None else _dev(y, torch.float64, self.n, "y")
        _check(load_library().spx_matmult(self.handle, _ptr(x), _ptr(y), _stream(stream)))
        return y

    def matmult_transpose(self, x: torch.Tensor, y: Optional[torch.Tensor] = None,
                          stream=None) -> torch.Tensor:
        _dev(x, torch.float64, self.n, "x")
        y = torch.empty_like(x) if y is None else _dev(y, torch.float64, self.n, "y")
        _check(load_library().spx_matmult_transpose(self.handle, _ptr(x), _ptr(y),
                                                    _stream(stream)))
        return y

    def spmm(self, X: torch.Tensor, Y: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if X.dim() != 2 or X.shape[0] != self.n:
            raise ValueError("X must be n x nrhs (row-major)")
        _dev(X, torch.float64, None, "X")
        nrhs = X.shape[1]
        Y = torch.empty_like(X) if Y is None else _dev(Y, torch.float64, self.n * nrhs, "Y")
        _check(load_library().spx_spmm(self.handle, nrhs, _ptr(X), nrhs, _ptr(Y), nrhs,
                                       _stream(stream)))
        return Y

    # -- solvers
    def _solve(self, fn, b, x, rtol, maxit, check_every, stream):
        _dev(b, torch.float64, self.n, "b")
        x = torch.zeros_like(b) if x is None else _dev(x, torch.float64, self.n, "x")
        it = ctypes.c_int64()
        rr = ctypes.c_double()
        rc = fn(self.handle, _ptr(b), _ptr(x), rtol, maxit, check_every, _stream(stream),
                ctypes.byref(it), ctypes.byref(rr))
        _check(rc, _SOLVER_OUTCOMES)
        return SolveResult(x, it.value, rr.value, rc)

    def cg_solve(self, b, x=None, rtol=1e-10, maxit=100000, check_every=20, stream=None):
        return self._solve(load_library().spx_cg_solve, b, x, rtol, maxit, check_every, stream)

    def cg_solve_noalloc(self, b, x, rtol=1e-10, maxit=100000, check_every=20, stream=None):
        """spx_cg_solve_noalloc: the same solve in the library's static
        scratch (n <= NOALLOC_MAX_ROWS).  x is required (in: x0, out: the
        solution), so that the call allocates nothing on this side either."""
        if x is None:
            raise ValueError("cg_solve_noalloc needs x (the call allocates nothing)")
        return self._solve(load_library().spx_cg_solve_noalloc, b, x, rtol, maxit, check_every,
                           stream)

    def cg_solve_transpose(self, b, x=None, rtol=1e-10, maxit=100000, check_every=20, stream=None):
        return self._solve(load_library().spx_cg_solve_transpose, b, x, rtol, maxit, check_every,
                           stream)

    def cg_solve_mixed(self, b, x=None, rtol_outer=1e-10, rtol_inner=1e-4, maxit_outer=100,
                       maxit_inner=100000, check_every=20, stream=None, early_exit=None):
        """FP32-inner / FP64-outer refinement.  ``early_exit`` (when not None)
        sets OPT_IR_EARLY_EXIT on the handle first: False runs every inner
        solve to rtol_inner, True also ends it at rtol_outer ||b|| / 2."""
        _dev(b, torch.float64, self.n, "b")
        if early_exit is not None:
            self.set_option(OPT_IR_EARLY_EXIT, 1 if early_exit else 0)
        x = torch.zeros_like(b) if x is None else _dev(x, torch.float64, self.n, "x")
        outer, inner = ctypes.c_int64(), ctypes.c_int64()
        rr = ctypes.c_double()
        rc = load_library().spx_cg_solve_mixed(self.handle, _ptr(b), _ptr(x), rtol_outer,
                                               rtol_inner, maxit_outer, maxit_inner, check_every,
                                               _stream(stream), ctypes.byref(outer),
                                               ctypes.byref(inner), ctypes.byref(rr))
        _check(rc, _SOLVER_OUTCOMES)
        return MixedResult(x, outer.value, inner.value, rr.value, rc)

    # -- reverse mode
    def sddmm(self, lam, u, G=None, stream=None):
        _dev(lam, torch.float64, self.n, "lam")
        _dev(u, torch.float64, self.n, "u")
        nnz = self.nnz
        G = torch.empty(nnz, dtype=torch.float64, device=self.device) if G is None else \
            _dev(G, torch.float64, nnz, "G")
        _check(load_library().spx_sddmm(self.handle, _ptr(lam), _ptr(u), _ptr(G), _stream(stream)))
        return G

    def coo_gather(self, G, grad_v=None, stream=None):
        _dev(G, torch.float64, self.nnz, "G")
        grad_v = torch.empty(self.ncoo, dtype=torch.float64, device=self.device) \
            if grad_v is None else _dev(grad_v, torch.float64, self.ncoo, "grad_v")
        _check(load_library().spx_coo_gather(self.handle, _ptr(G), _ptr(grad_v), _stream(stream)))
        return grad_v

    def coo_gather_blocks(self, G, w, block: int, grad_e=None, stream=None):
        _dev(G, torch.float64, self.nnz, "G")
        _dev(w, torch.float64, self.ncoo, "w")
        nb = self.ncoo // block if block > 0 else 0
        grad_e = torch.empty(nb, dtype=torch.float64, device=self.device) \
            if grad_e is None else _dev(grad_e, torch.float64, nb, "grad_e")
        _check(load_library().spx_coo_gather_blocks(self.handle, _ptr(G), _ptr(w), block,
                                                    _ptr(grad_e), _stream(stream)))
        return grad_e

    # -- options
    def set_option(self, option: int, value: int) -> None:
        _check(load_library().spx_set_option(self.handle, option, value))

    def get_option(self, option: int) -> int:
        v = ctypes.c_int64()
        _check(load_library().spx_get_option(self.handle, option, ctypes.byref(v)))
        return v.value

    def get_profile(self) -> dict:
        out = {}
        for k, name in enumerate(PROFILE_KINDS):
            ms, cnt = ctypes.c_double(), ctypes.c_int64()
            _check(load_library().spx_get_profile(self.handle, k, ctypes.byref(ms),
                                                  ctypes.byref(cnt)))
            out[name] = (ms.value, cnt.value)
        return out

    def reset_profile(self) -> None:
        _check(load_library().spx_reset_profile(self.handle))


def coo_preallocate(n: int, i: torch.Tensor, j: torch.Tensor, stream=None) -> Matrix:
    """Symbolic COO stage on the GPU (paper Sec. 5); returns a Matrix."""
    ncoo = i.numel()
    _dev(i, torch.int32, None, "i")
    _dev(j, torch.int32, ncoo, "j")
    h = ctypes.c_void_p()
    _check(load_library().spx_coo_preallocate(n, ncoo, _ptr(i), _ptr(j), _stream(stream),
                                              ctypes.byref(h)))
    return Matrix(h, n, ncoo, i.device)


class SplitMatrix:
    """One rank's rows [row_lo, row_hi) of an n_global x n_global matrix as a
    diagonal block and a compressed off-diagonal block (spx_split_*)."""

    def __init__(self, n_global: int, row_lo: int, row_hi: int, i: torch.Tensor, j: torch.Tensor,
                 stream=None):
        ncoo = i.numel()
        _dev(i, torch.int32, None, "i")
        _dev(j, torch.int32, ncoo, "j")
        self._h = None
        h = ctypes.c_void_p()
        _check(load_library().spx_split_preallocate(n_global, row_lo, row_hi, ncoo, _ptr(i),
                                                    _ptr(j), _stream(stream), ctypes.byref(h)))
        self._h = h
        self.n_global, self.row_lo, self.row_hi, self.ncoo = n_global, row_lo, row_hi, ncoo
        self.device = i.device
        rows, ng, nro, nrem = (ctypes.c_int64() for _ in range(4))
        _check(load_library().spx_split_get_info(h, ctypes.byref(rows), ctypes.byref(ng),
                                                 ctypes.byref(nro), ctypes.byref(nrem)))
        self.rows, self.nghost, self.nrows_offdiag, self.nremote = (rows.value, ng.value,
                                                                    nro.value, nrem.value)
        d, o = ctypes.c_void_p(), ctypes.c_void_p()
        _check(load_library().spx_split_blocks(h, ctypes.byref(d), ctypes.byref(o)))
        self.diag = Matrix(d, self.rows, ncoo, self.device, owner=self)
        self.offdiag = Matrix(o, max(self.nrows_offdiag, self.nghost, 1), ncoo, self.device,
                              owner=self)

    def destroy(self) -> None:
        if self._h:
            self.diag.destroy()
            self.offdiag.destroy()
            _check(load_library().spx_split_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        if not self._h:
            raise RuntimeError("split matrix has been destroyed")
        return self._h

    def set_values_coo(self, v: torch.Tensor, mode: int = INSERT_VALUES, stream=None) -> None:
        _dev(v, torch.float64, self.ncoo, "v")
        _check(load_library().spx_split_set_values_coo(self.handle, _ptr(v), mode, _stream(stream)))

    def maps(self, stream=None):
        """(garray, orows): the ghost columns' global numbers and the local rows
        of the off-diagonal block."""
        garray = torch.empty(self.nghost, dtype=torch.int32, device=self.device)
        orows = torch.empty(self.nrows_offdiag, dtype=torch.int32, device=self.device)
        _check(load_library().spx_split_get_maps(self.handle, _ptr(garray), _ptr(orows),
                                                 _stream(stream)))
        return garray, orows

    def gather_ghosts(self, x_global: torch.Tensor, x_ghost=None, stream=None) -> torch.Tensor:
        _dev(x_global, torch.float64, self.n_global, "x_global")
        x_ghost = torch.empty(self.nghost, dtype=torch.float64, device=self.device) \
            if x_ghost is None else _dev(x_ghost, torch.float64, self.nghost, "x_ghost")
        _check(load_library().spx_split_gather_ghosts(self.handle, _ptr(x_global), _ptr(x_ghost),
                                                      _stream(stream)))
        return x_ghost

    def matmult(self, x_local: torch.Tensor, x_ghost: torch.Tensor, y=None,
                stream=None) -> torch.Tensor:
        _dev(x_local, torch.float64, self.rows, "x_local")
        _dev(x_ghost, torch.float64, self.nghost, "x_ghost")
        y = torch.empty_like(x_local) if y is None else _dev(y, torch.float64, self.rows, "y")
        _check(load_library().spx_split_matmult(self.handle, _ptr(x_local), _ptr(x_ghost), _ptr(y),
                                                _stream(stream)))
        return y


def split_preallocate(n_global: int, row_lo: int, row_hi: int, i: torch.Tensor, j: torch.Tensor,
                      stream=None) -> SplitMatrix:
    """Rows [row_lo, row_hi) of the COO stream as diagonal and off-diagonal
    blocks (paper Sec. 5)."""
    return SplitMatrix(n_global, row_lo, row_hi, i, j, stream)


class BatchTuning(ctypes.Structure):
    """Launch shape of the batched solver (mirrors spx_batch_tuning)."""

    _fields_ = [("blocks", ctypes.c_int32), ("rows_per_tile", ctypes.c_int32),
                ("weight_exponent", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("persistent", ctypes.c_int32)]


class Batch:
    """Several assembled matrices solved together by one persistent launch."""

    def __init__(self, mats: Sequence[Matrix], stream=None):
        self.mats = list(mats)
        arr = (ctypes.c_void_p * len(self.mats))(*[m.handle for m in self.mats])
        h = ctypes.c_void_p()
        _check(load_library().spx_batch_create(len(self.mats), arr, _stream(stream),
                                               ctypes.byref(h)))
        self._h = h
        tot = ctypes.c_int64()
        _check(load_library().spx_batch_total_rows(self._h, ctypes.byref(tot)))
        self.total = tot.value
        self.offsets = [0]
        for m in self.mats:
            self.offsets.append(self.offsets[-1] + m.n)

    def destroy(self):
        if self._h:
            _check(load_library().spx_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def _solve(self, fn, b, x, rtol, maxit, blocks, rows_per_tile, weight_exponent, check_every,
               stream, persistent=0):
        _dev(b, torch.float64, self.total, "b")
        x = torch.zeros_like(b) if x is None else _dev(x, torch.float64, self.total, "x")
        ns = len(self.mats)
        iters = (ctypes.c_int64 * ns)()
        rel = (ctypes.c_double * ns)()
        tune = BatchTuning(blocks, rows_per_tile, weight_exponent, check_every, persistent)
        rc = fn(self._h, _ptr(b), _ptr(x), rtol, maxit,
                ctypes.cast(ctypes.byref(tune), ctypes.c_void_p), _stream(stream),
                ctypes.cast(iters, _pi64), ctypes.cast(rel, _pd))
        _check(rc, _SOLVER_OUTCOMES)
        return x, list(iters), list(rel), rc

    def batch_cg(self, b, x=None, rtol=1e-8, maxit=100000, blocks=0, rows_per_tile=0,
                 weight_exponent=1.0, check_every=20, stream=None, persistent=0):
        """Jacobi-CG on every system (SPD systems).  persistent: 1 for one
        launch in which each workgroup solves whole systems taken from a
        queue, -1 for one launch per phase, 0 to let the library choose."""
        return self._solve(load_library().spx_batch_cg, b, x, rtol, maxit, blocks, rows_per_tile,
                           weight_exponent, check_every, stream, persistent)

    def batch_bicg(self, b, x=None, rtol=1e-8, maxit=100000, blocks=0, rows_per_tile=0,
                   weight_exponent=1.0, check_every=20, stream=None, persistent=0):
        """Jacobi-preconditioned BiCG on every system (iterations: BiCG steps);
        persistent as in batch_cg."""
        return self._solve(load_library().spx_batch_bicg, b, x, rtol, maxit, blocks,
                           rows_per_tile, weight_exponent, check_every, stream, persistent)

    def batch_tfqmr(self, b, x=None, rtol=1e-8, maxit=100000, blocks=0, rows_per_tile=0,
                    weight_exponent=1.0, check_every=20, stream=None, persistent=0):
        """Right-Jacobi TFQMR on every system (iterations: half-steps, one
        product with A each; maxit counts half-steps, check_every full
        iterations of two half-steps); persistent as in batch_cg."""
        return self._solve(load_library().spx_batch_tfqmr, b, x, rtol, maxit, blocks,
                           rows_per_tile, weight_exponent, check_every, stream, persistent)


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)
_hooks = []  # keeps the installed callbacks alive


def use_torch_allocator(enable: bool = True) -> None:
    """Routes the library's device allocations through PyTorch's caching
    allocator (on the current device and stream at allocation time), or back
    to hipMalloc with enable=False.  Blocks are returned to whichever
    allocator made them."""
    lib = load_library()
    if not enable:
        _check(lib.spx_set_allocator(None, None, None))
        return

    def _alloc(nbytes, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                      torch.cuda.current_stream())
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC_FN(_alloc), _FREE_FN(_free)
    _hooks.append((a, f))
    _check(lib.spx_set_allocator(ctypes.cast(a, ctypes.c_void_p), ctypes.cast(f, ctypes.c_void_p),
                                 None))


def stream_copy(x: torch.Tensor, y: torch.Tensor, stream=None) -> torch.Tensor:
    """y = x with the library's bandwidth-reference copy kernel."""
    _dev(x, torch.float64, None, "x")
    _dev(y, torch.float64, x.numel(), "y")
    _check(load_library().spx_stream_copy(_ptr(x), _ptr(y), x.numel(), _stream(stream)))
    return y


def stream_sum(x: torch.Tensor, partials: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Per-workgroup sums of x (2048 of them) with the bandwidth-reference read kernel."""
    _dev(x, torch.float64, None, "x")
    if partials is None:
        partials = torch.empty(2048, dtype=torch.float64, device=x.device)
    _dev(partials, torch.float64, 2048, "partials")
    _check(load_library().spx_stream_sum(_ptr(x), x.numel(), _ptr(partials), _stream(stream)))
    return partials


def batch_create(mats: Sequence[Matrix], stream=None) -> Batch:
    return Batch(mats, stream)


class Lbfgs:
    """Limited-memory BFGS history on the GPU (paper Sec. 8): update with
    pairs (s, y), apply p = H_k g in the intermediate dense form."""

    def __init__(self, n: int, m: int, stream=None):
        h = ctypes.c_void_p()
        _check(load_library().spx_lbfgs_create(n, m, _stream(stream), ctypes.byref(h)))
        self._h, self.n, self.m = h, n, m

    def update(self, s, y, stream=None) -> None:
        _dev(s, torch.float64, self.n, "s")
        _dev(y, torch.float64, self.n, "y")
        _check(load_library().spx_lbfgs_update(self._h, _ptr(s), _ptr(y), _stream(stream)))

    def apply(self, g, h0=None, p=None, stream=None):
        _dev(g, torch.float64, self.n, "g")
        if h0 is not None:
            _dev(h0, torch.float64, self.n, "h0")
        p = torch.empty_like(g) if p is None else _dev(p, torch.float64, self.n, "p")
        _check(load_library().spx_lbfgs_apply(self._h, _ptr(g), _ptr(h0) if h0 is not None else None,
                                              _ptr(p), _stream(stream)))
        return p

    def update_apply(self, s, y, g, h0=None, p=None, stream=None):
        """update(s, y) then apply(g, h0, p), with S^T g taken in the
        update's pass over S (the same bits as the two calls)."""
        _dev(s, torch.float64, self.n, "s")
        _dev(y, torch.float64, self.n, "y")
        _dev(g, torch.float64, self.n, "g")
        if h0 is not None:
            _dev(h0, torch.float64, self.n, "h0")
        p = torch.empty_like(g) if p is None else _dev(p, torch.float64, self.n, "p")
        _check(load_library().spx_lbfgs_update_apply(self._h, _ptr(s), _ptr(y), _ptr(g),
                                                     _ptr(h0) if h0 is not None else None,
                                                     _ptr(p), _stream(stream)))
        return p

    def reset(self) -> None:
        _check(load_library().spx_lbfgs_reset(self._h))

    @property
    def count(self) -> int:
        c = ctypes.c_int32()
        _check(load_library().spx_lbfgs_get_info(self._h, None, None, ctypes.byref(c)))
        return c.value

    def destroy(self):
        if self._h:
            _check(load_library().spx_lbfgs_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def lbfgs_create(n: int, m: int, stream=None) -> Lbfgs:
    return Lbfgs(n, m, stream)


class CooVector:
    """A COO vector pattern on the GPU (paper Sec. 5, VecSetPreallocationCOO)."""

    def __init__(self, handle, n: int, ncoo: int, device):
        self._h = handle
        self.n = n
        self.ncoo = ncoo
        self.device = device

    def destroy(self):
        if self._h:
            _check(load_library().spx_vec_coo_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def get_info(self):
        n, nu, nv, nc = (ctypes.c_int64() for _ in range(4))
        _check(load_library().spx_vec_coo_get_info(self._h, ctypes.byref(n), ctypes.byref(nu),
                                                   ctypes.byref(nv), ctypes.byref(nc)))
        return {"n": n.value, "nunique": nu.value, "nvalid": nv.value, "ncoo": nc.value}

    def set_values_coo(self, v, x, mode: int = INSERT_VALUES, stream=None):
        _dev(v, torch.float64, self.ncoo, "v")
        _dev(x, torch.float64, self.n, "x")
        _check(load_library().spx_vec_set_values_coo(self._h, _ptr(v), mode, _ptr(x),
                                                     _stream(stream)))
        return x


def vec_coo_preallocate(n: int, i: torch.Tensor, stream=None) -> CooVector:
    """Symbolic COO stage of a vector on the GPU (paper Sec. 5)."""
    _dev(i, torch.int32, None, "i")
    h = ctypes.c_void_p()
    _check(load_library().spx_vec_coo_preallocate(n, i.numel(), _ptr(i), _stream(stream),
                                                  ctypes.byref(h)))
    return CooVector(h, n, i.numel(), i.device)


def version() -> str:
    return load_library().spx_version().decode()
