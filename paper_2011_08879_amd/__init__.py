"""Python binding of libgko_mi355x.so (the C ABI declared in include/gko.h).

Argument marshalling only: every step runs in the library's HIP kernels.
PyTorch supplies device memory (its caching allocator is installed as the
library's allocator) and the current stream.  Importing this module does not
need a GPU; creating a Context does.  If the shared library has not been
built, importing raises ImportError -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgko_mi355x.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libgko_mi355x.so is not built; run `python paper_2011_08879_amd/build.py` "
                      "(or __graft_entry__.build())")

# torch ships its own HIP runtime (same soname as /opt/rocm's).  Loading torch
# first makes the library bind to that already-loaded runtime, so streams and
# device pointers handed over by torch belong to the runtime the library uses.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ----------------------------------------------------------------------------- enums
OK, ERR_INVALID_ARG, ERR_DIM_MISMATCH, ERR_UNSUPPORTED, ERR_ALLOC, ERR_HIP = 0, 1, 2, 3, 4, 5
ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NOT_SPD = 6, 7, 8
F64, F32 = 0, 1
I32, I64 = 0, 1
FORMATS = {"csr": 0, "csr_merge": 1, "coo": 2, "ell": 3, "hybrid": 4, "auto": 5, "sellp": 6}
FORMAT_NAMES = {v: k for k, v in FORMATS.items()}
PREC_FP64, PREC_MIXED_IR = 0, 1
PRECOND_NONE, PRECOND_BLOCK_JACOBI = 0, 1

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_f64 = ctypes.c_double
_st = ctypes.c_int


class _MatrixDesc(ctypes.Structure):
    _fields_ = [("format", _i32), ("dtype", _i32), ("n_rows", _i64), ("n_cols", _i64),
                ("nnz", _i64), ("ell_width", _i64), ("ell_ld", _i64), ("coo_nnz", _i64),
                ("stored_bytes", _i64), ("csr_kernel", _i32), ("max_row_len", _i32),
                ("csr_long_rows", _i64), ("sellp_slices", _i64), ("sellp_slots", _i64),
                ("sellp_slice", _i32), ("csr_row_lanes", _i32), ("sellp_wide_slices", _i64)]


class SolverOpts(ctypes.Structure):
    _fields_ = [("precision", _i32), ("precond", _i32), ("block_size", _i32),
                ("check_every", _i32), ("inner_tol", _f64), ("max_inner", _i32),
                ("max_outer", _i32), ("single_workgroup", _i32), ("krylov_dim", _i32),
                ("graphs", _i32)]


class _SolveInfo(ctypes.Structure):
    _fields_ = [("status", _i32), ("iterations", _i32), ("outer_iterations", _i32),
                ("restarts", _i32), ("rel_residual", _f64), ("true_rel_residual", _f64),
                ("seconds", _f64), ("setup_seconds", _f64), ("reorthogonalized", _i32),
                ("pad", _i32)]


ALLOC_FN = ctypes.CFUNCTYPE(_vp, ctypes.c_size_t, _vp, _vp)
DEALLOC_FN = ctypes.CFUNCTYPE(None, _vp, _vp, _vp)

_SIGS = {
    "gko_context_create": [_vp, ctypes.POINTER(_vp)],
    "gko_context_destroy": [_vp],
    "gko_context_set_stream": [_vp, _vp],
    "gko_context_set_allocator": [_vp, ALLOC_FN, DEALLOC_FN, _vp],
    "gko_matrix_create_csr": [_vp, _i64, _i64, _i64, _st, _vp, _st, _vp, _vp, ctypes.POINTER(_vp)],
    "gko_matrix_destroy": [_vp],
    "gko_matrix_clone": [_vp, ctypes.POINTER(_vp)],
    "gko_matrix_describe": [_vp, ctypes.POINTER(_MatrixDesc)],
    "gko_matrix_export_csr": [_vp, _vp, _vp, _vp],
    "gko_matrix_export_storage": [_vp, _vp, _vp, _vp, _vp, _vp],
    "gko_matrix_export_sellp": [_vp, _vp, _vp, _vp, _vp],
    "gko_spmv": [_vp, _f64, _vp, _f64, _vp],
    "gko_convert": [_vp, _st],
    "gko_dot": [_vp, _st, _i64, _vp, _vp, _vp],
    "gko_norm2": [_vp, _st, _i64, _vp, _vp],
    "gko_stream": [_vp, _st, _i64, _vp, _vp, _f64, _vp],
    "gko_gather_probe": [_vp, _i64, _vp, _i64, _vp, _vp],
    "gko_context_set_solver_opts": [_vp, ctypes.POINTER(SolverOpts)],
    "gko_context_get_solver_opts": [_vp, ctypes.POINTER(SolverOpts)],
    "gko_context_get_solve_info": [_vp, ctypes.POINTER(_SolveInfo)],
    "gko_cg_solve": [_vp, _vp, _vp, _f64, _i32],
    "gko_cg_solve_noalloc": [_vp, _vp, _vp, _f64, _i32],
    "gko_matrix_features": [_vp, ctypes.POINTER(ctypes.c_float)],
    "gko_autotune_format": [_vp, ctypes.POINTER(_st), ctypes.POINTER(ctypes.c_float)],
    "gko_select_format": [_vp, _vp, ctypes.POINTER(_st), ctypes.POINTER(ctypes.c_float)],
    "gko_context_set_selector": [_vp, _vp],
    "gko_mlp_create": [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_vp)],
    "gko_mlp_destroy": [_vp],
    "gko_mlp_get_params": [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
    "gko_mlp_fit_normalization": [_vp, _i64, _vp],
    "gko_mlp_forward": [_vp, _i64, _vp, _vp],
    "gko_mlp_loss_grad": [_vp, _i64, _vp, _vp, _vp, _vp, _vp],
    "gko_mlp_train": [_vp, _i64, _vp, _vp, _vp, _i32, ctypes.c_float, _vp],
    "gko_mlp_save": [_vp, ctypes.c_char_p],
    "gko_mlp_load": [_vp, ctypes.c_char_p, ctypes.POINTER(_vp)],
    "gko_batch_create_csr": [_vp, _i64, _vp, _vp, _vp, _vp, _vp, _st, ctypes.POINTER(_vp)],
    "gko_batch_destroy": [_vp],
    "gko_batch_cg_solve": [_vp, _vp, _vp, _f64, _i32, _vp, _vp],
    "gko_batch_set_block": [_vp, _i32],
    "gko_batch_get_block": [_vp, ctypes.POINTER(_i32)],
    "gko_batch_launch_info": [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64)],
    "gko_batch_set_lds_mode": [_vp, _i32],
    "gko_batch_get_lds_mode": [_vp, ctypes.POINTER(_i32)],
    "gko_batch_autotune": [_vp, _vp, _vp, _f64, _i32, _vp, _vp, ctypes.POINTER(_i32),
                           ctypes.POINTER(ctypes.c_float)],
    "gko_bicgstab_solve": [_vp, _vp, _vp, _f64, _i32],
    "gko_fcg_solve": [_vp, _vp, _vp, _f64, _i32],
    "gko_pipecg_solve": [_vp, _vp, _vp, _f64, _i32],
    "gko_cgs_solve": [_vp, _vp, _vp, _f64, _i32],
    "gko_gmres_solve": [_vp, _vp, _vp, _f64, _i32],
}
for _name, _args in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _st
_lib.gko_last_error.argtypes = []
_lib.gko_last_error.restype = ctypes.c_char_p
_lib.gko_status_string.argtypes = [_st]
_lib.gko_status_string.restype = ctypes.c_char_p

EXPORTED = tuple(_SIGS) + ("gko_last_error", "gko_status_string")


class GkoError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (status_string(status), status, message))
        self.status = status


def status_string(status: int) -> str:
    return _lib.gko_status_string(status).decode()


def last_error() -> str:
    return _lib.gko_last_error().decode()


def _check(status: int):
    if status != OK:
        raise GkoError(status, last_error())


def _torch():
    import torch
    return torch


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _vec(t, n: int, dtype, name: str):
    """The C-ABI takes bare device pointers, so the binding checks what it can
    see: `t` is a contiguous CUDA tensor of `dtype` with at least n elements."""
    if t is None:
        raise ValueError("%s: a device tensor is required" % name)
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("%s: expected a contiguous CUDA tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s: expected %s, got %s" % (name, dtype, t.dtype))
    if t.numel() < n:
        raise ValueError("%s: %d elements, at least %d needed" % (name, t.numel(), n))


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return F64
    if t.dtype == torch.float32:
        return F32
    raise TypeError("values must be float64 or float32, got %s" % t.dtype)


# ----------------------------------------------------------------------------- context
class Context:
    """Binds the library to the current torch stream and torch's caching allocator."""

    def __init__(self, device: int | None = None, use_torch_allocator: bool = True):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the library has no CPU path")
        if device is not None:
            torch.cuda.set_device(device)
        self.device = torch.cuda.current_device()
        h = _vp()
        _check(_lib.gko_context_create(_vp(torch.cuda.current_stream().cuda_stream),
                                       ctypes.byref(h)))
        self.handle = h
        self._cbs = None
        if use_torch_allocator:
            dev = self.device

            def _alloc(nbytes, stream, user):
                try:
                    return torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream or 0)
                except Exception:  # surfaced to C as NULL -> GKO_ERR_ALLOC
                    return None

            def _dealloc(p, stream, user):
                torch.cuda.caching_allocator_delete(p)

            self._cbs = (ALLOC_FN(_alloc), DEALLOC_FN(_dealloc))
            _check(_lib.gko_context_set_allocator(h, self._cbs[0], self._cbs[1], None))

    def sync_stream(self):
        """Rebind to torch's current stream (call after switching streams)."""
        torch = _torch()
        _check(_lib.gko_context_set_stream(self.handle,
                                           _vp(torch.cuda.current_stream().cuda_stream)))

    @property
    def stream(self) -> int:
        return _torch().cuda.current_stream().cuda_stream

    def set_solver_opts(self, precision: int = PREC_FP64, precond: int = PRECOND_NONE,
                        block_size: int = 8, check_every: int = 16, inner_tol: float = 1e-5,
                        max_inner: int = 1000, max_outer: int = 20, single_workgroup: int = 1,
                        krylov_dim: int = 30, graphs: int = 1):
        o = SolverOpts(precision, precond, block_size, check_every, inner_tol, max_inner, max_outer,
                       single_workgroup, krylov_dim, graphs)
        _check(_lib.gko_context_set_solver_opts(self.handle, ctypes.byref(o)))

    def solver_opts(self) -> dict:
        o = SolverOpts()
        _check(_lib.gko_context_get_solver_opts(self.handle, ctypes.byref(o)))
        return {f: getattr(o, f) for f, _ in SolverOpts._fields_}

    def solve_info(self) -> dict:
        i = _SolveInfo()
        _check(_lib.gko_context_get_solve_info(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _SolveInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            _lib.gko_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default_ctx: Context | None = None


def default_context() -> Context:
    global _default_ctx
    if _default_ctx is None:
        _default_ctx = Context()
    return _default_ctx


# ----------------------------------------------------------------------------- matrices
@dataclass
class Desc:
    format: str
    dtype: str
    n_rows: int
    n_cols: int
    nnz: int
    ell_width: int
    ell_ld: int
    coo_nnz: int
    stored_bytes: int
    csr_kernel: int      # CSR: 0 row-per-thread (LDS-staged), else subwarp lanes; -1 otherwise
    max_row_len: int
    csr_long_rows: int
    sellp_slices: int    # SELLP: number of slices, else 0
    sellp_slots: int     # SELLP: slots including padding, else 0
    sellp_slice: int     # SELLP: rows per slice, else 0
    sellp_wide_slices: int  # SELLP: slices summed by column chunks, else 0
    csr_row_lanes: int = 0  # CSR row-per-thread kernel: lanes per row, else 0


class Matrix:
    """A sparse matrix owned by the library (device storage, any format)."""

    def __init__(self, handle, ctx: Context):
        self.handle = handle
        self.ctx = ctx
        self._dims = None

    def _shape_dtype(self):
        if self._dims is None:
            d = self.describe()
            torch = _torch()
            self._dims = (d.n_rows, d.n_cols, torch.float64 if d.dtype == "f64" else torch.float32)
        return self._dims

    @classmethod
    def from_csr(cls, row_ptr, col, val, n_cols: int | None = None, ctx: Context | None = None,
                 dtype=None):
        """Create from CSR arrays (numpy or torch, host or device); they are copied."""
        torch = _torch()
        ctx = ctx or default_context()
        dev = torch.device("cuda", ctx.device)

        def dev_tensor(a, dt):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=dev, dtype=dt).contiguous()

        rp_t = row_ptr if isinstance(row_ptr, torch.Tensor) else torch.from_numpy(
            np.ascontiguousarray(row_ptr))
        itype = I64 if rp_t.dtype == torch.int64 else I32
        rp = dev_tensor(rp_t, torch.int64 if itype == I64 else torch.int32)
        ci = dev_tensor(col, torch.int32)
        vdt = dtype or (val.dtype if isinstance(val, torch.Tensor) else
                        (torch.float32 if np.asarray(val).dtype == np.float32 else torch.float64))
        va = dev_tensor(val, vdt)
        n = rp.numel() - 1
        m = n if n_cols is None else int(n_cols)
        h = _vp()
        _check(_lib.gko_matrix_create_csr(ctx.handle, n, m, ci.numel(), _dtype_code(va), _ptr(rp),
                                          itype, _ptr(ci), _ptr(va), ctypes.byref(h)))
        return cls(h, ctx)

    def describe(self) -> Desc:
        d = _MatrixDesc()
        _check(_lib.gko_matrix_describe(self.handle, ctypes.byref(d)))
        return Desc(FORMAT_NAMES[d.format], "f64" if d.dtype == F64 else "f32", d.n_rows,
                    d.n_cols, d.nnz, d.ell_width, d.ell_ld, d.coo_nnz, d.stored_bytes,
                    d.csr_kernel, d.max_row_len, d.csr_long_rows, d.sellp_slices, d.sellp_slots,
                    d.sellp_slice, d.sellp_wide_slices, d.csr_row_lanes)

    @property
    def shape(self):
        d = self.describe()
        return d.n_rows, d.n_cols

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.describe().dtype == "f64" else torch.float32

    def convert(self, fmt: str) -> "Matrix":
        _check(_lib.gko_convert(self.handle, FORMATS[fmt]))
        return self

    def clone(self) -> "Matrix":
        h = _vp()
        _check(_lib.gko_matrix_clone(self.handle, ctypes.byref(h)))
        return Matrix(h, self.ctx)

    def export_csr(self):
        torch = _torch()
        d = self.describe()
        dev = torch.device("cuda", self.ctx.device)
        rp = torch.empty(d.n_rows + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(d.nnz, dtype=torch.int32, device=dev)
        va = torch.empty(d.nnz, dtype=self.torch_dtype, device=dev)
        _check(_lib.gko_matrix_export_csr(self.handle, _ptr(rp), _ptr(ci), _ptr(va)))
        return rp, ci, va

    def export_storage(self) -> dict:
        """Raw stored arrays of ELL / COO / HYBRID formats (for layout checks)."""
        torch = _torch()
        d = self.describe()
        dev = torch.device("cuda", self.ctx.device)
        out = {}
        ec = ev = cr = cc = cv = None
        if d.format in ("ell", "hybrid"):
            ec = torch.empty(d.ell_width * d.ell_ld, dtype=torch.int32, device=dev)
            ev = torch.empty(d.ell_width * d.ell_ld, dtype=self.torch_dtype, device=dev)
            out.update(ell_col=ec, ell_val=ev, K=d.ell_width, ld=d.ell_ld)
        if d.format in ("coo", "hybrid"):
            cr = torch.empty(d.coo_nnz, dtype=torch.int32, device=dev)
            cc = torch.empty(d.coo_nnz, dtype=torch.int32, device=dev)
            cv = torch.empty(d.coo_nnz, dtype=self.torch_dtype, device=dev)
            out.update(coo_row=cr, coo_col=cc, coo_val=cv)
        _check(_lib.gko_matrix_export_storage(self.handle, _ptr(ec), _ptr(ev), _ptr(cr), _ptr(cc),
                                              _ptr(cv)))
        return out

    def export_sellp(self) -> dict:
        """Raw SELL-P arrays: slice offsets (int64), widths, slot columns and values."""
        torch = _torch()
        d = self.describe()
        dev = torch.device("cuda", self.ctx.device)
        sets = torch.empty(d.sellp_slices + 1, dtype=torch.int64, device=dev)
        widths = torch.empty(d.sellp_slices, dtype=torch.int32, device=dev)
        col = torch.empty(d.sellp_slots, dtype=torch.int32, device=dev)
        val = torch.empty(d.sellp_slots, dtype=self.torch_dtype, device=dev)
        _check(_lib.gko_matrix_export_sellp(self.handle, _ptr(sets), _ptr(widths), _ptr(col),
                                            _ptr(val)))
        return dict(sets=sets, widths=widths, col=col, val=val, slice=d.sellp_slice)

    def close(self):
        if getattr(self, "handle", None):
            _lib.gko_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- operations
def spmv(A: Matrix, alpha: float, x, beta: float, y):
    """y <- alpha A x + beta y (asynchronous on the current stream)."""
    n, m, dt = A._shape_dtype()
    _vec(x, m, dt, "x")
    _vec(y, n, dt, "y")
    _check(_lib.gko_spmv(A.handle, alpha, _ptr(x), beta, _ptr(y)))
    return y


def convert(A: Matrix, fmt: str) -> Matrix:
    return A.convert(fmt)


def dot(x, y, ctx: Context | None = None):
    """x.y accumulated in FP64; returns a 0-d float64 device tensor."""
    torch = _torch()
    _vec(x, 0, x.dtype, "x")
    _vec(y, x.numel(), x.dtype, "y")
    ctx = ctx or default_context()
    out = torch.empty((), dtype=torch.float64, device=x.device)
    _check(_lib.gko_dot(ctx.handle, _dtype_code(x), x.numel(), _ptr(x), _ptr(y), _ptr(out)))
    return out


def norm2(x, ctx: Context | None = None):
    torch = _torch()
    _vec(x, 0, x.dtype, "x")
    ctx = ctx or default_context()
    out = torch.empty((), dtype=torch.float64, device=x.device)
    _check(_lib.gko_norm2(ctx.handle, _dtype_code(x), x.numel(), _ptr(x), _ptr(out)))
    return out


STREAM_COPY, STREAM_TRIAD = 0, 1


def stream(op: int, a, c, b=None, s: float = 0.0, ctx: Context | None = None):
    """Bandwidth probe on float64 device tensors: COPY c = a, TRIAD c = a + s b."""
    torch = _torch()
    _vec(a, 0, torch.float64, "a")
    _vec(c, a.numel(), torch.float64, "c")
    if op == STREAM_TRIAD:
        _vec(b, a.numel(), torch.float64, "b")
    ctx = ctx or default_context()
    _check(_lib.gko_stream(ctx.handle, op, a.numel(), _ptr(a), _ptr(b), s, _ptr(c)))
    return c


def _solve(fn, A: Matrix, b, x, tol: float, maxit: int, raise_on_failure: bool):
    torch = _torch()
    n = A._shape_dtype()[0]
    _vec(b, n, torch.float64, "b")
    _vec(x, n, torch.float64, "x")
    st = fn(A.handle, _ptr(b), _ptr(x), tol, maxit)
    err = last_error() if st != OK else ""   # read before the next call clears it
    info = A.ctx.solve_info()
    info["status"] = st
    info["status_name"] = status_string(st)
    info["error"] = err
    if st != OK and raise_on_failure:
        raise GkoError(st, err)
    return info


def gather_probe(x, idx, y, ctx: Context | None = None):
    """y[i] = x[idx[i]] (FP64 x and y, int32 idx; CUDA tensors): the random-gather ceiling."""
    torch = _torch()
    _vec(x, 1, torch.float64, "x")
    _vec(idx, 0, torch.int32, "idx")
    _vec(y, idx.numel(), torch.float64, "y")
    ctx = ctx or default_context()
    _check(_lib.gko_gather_probe(ctx.handle, idx.numel(), _ptr(x), x.numel(), _ptr(idx), _ptr(y)))
    return y


def cg(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000, raise_on_failure: bool = False):
    """(P)CG, options from the context.  x: initial guess in, solution out.  Returns solve info."""
    return _solve(_lib.gko_cg_solve, A, b, x, tol, maxit, raise_on_failure)


CG_NOALLOC_MAX_ROWS = 2752448   # GKO_CG_NOALLOC_MAX_ROWS
BATCH_LDS_MODES = ("all", "direction", "waves")   # gko_batch_lds


def cg_noalloc(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000,
               raise_on_failure: bool = False):
    """cg() without device allocation: FP64, no preconditioner, at most
    CG_NOALLOC_MAX_ROWS rows; work buffers in the library's static scratch."""
    return _solve(_lib.gko_cg_solve_noalloc, A, b, x, tol, maxit, raise_on_failure)


def bicgstab(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000,
             raise_on_failure: bool = False):
    return _solve(_lib.gko_bicgstab_solve, A, b, x, tol, maxit, raise_on_failure)


def fcg(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000, raise_on_failure: bool = False):
    """Flexible (P)CG (Polak-Ribiere beta), the same options as cg()."""
    return _solve(_lib.gko_fcg_solve, A, b, x, tol, maxit, raise_on_failure)


def pipecg(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000,
           raise_on_failure: bool = False):
    """Pipelined (P)CG (Ghysels-Vanroose): one reduction per iteration; options as cg()."""
    return _solve(_lib.gko_pipecg_solve, A, b, x, tol, maxit, raise_on_failure)


def cgs(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000, raise_on_failure: bool = False):
    """Unpreconditioned CGS (FP64)."""
    return _solve(_lib.gko_cgs_solve, A, b, x, tol, maxit, raise_on_failure)


def gmres(A: Matrix, b, x, tol: float = 1e-10, maxit: int = 10000,
          raise_on_failure: bool = False):
    """Restarted GMRES(m), m = the context's krylov_dim option (FP64, unpreconditioned).
    Solve info: iterations = Arnoldi steps, outer_iterations = cycles."""
    return _solve(_lib.gko_gmres_solve, A, b, x, tol, maxit, raise_on_failure)


# ----------------------------------------------------------------------------- batched CG
class Batch:
    """Many small independent systems solved by one persistent kernel launch."""

    def __init__(self, row_off, nnz_off, row_ptr_local, col, val, ctx: Context | None = None,
                 dtype=None):
        torch = _torch()
        self.ctx = ctx or default_context()
        dev = torch.device("cuda", self.ctx.device)

        def d(a, dt):
            t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
            return t.to(device=dev, dtype=dt).contiguous()

        ro, no = d(row_off, torch.int64), d(nnz_off, torch.int64)
        rp, ci = d(row_ptr_local, torch.int32), d(col, torch.int32)
        va = d(val, dtype or torch.float64)
        self.nsys = ro.numel() - 1
        self.rows = int(ro[-1].item()) if self.nsys > 0 else 0
        h = _vp()
        _check(_lib.gko_batch_create_csr(self.ctx.handle, self.nsys, _ptr(ro), _ptr(no), _ptr(rp),
                                         _ptr(ci), _ptr(va), _dtype_code(va), ctypes.byref(h)))
        self.handle = h

    @property
    def block(self) -> int:
        b = _i32()
        _check(_lib.gko_batch_get_block(self.handle, ctypes.byref(b)))
        return b.value

    @block.setter
    def block(self, v: int):
        _check(_lib.gko_batch_set_block(self.handle, v))

    def launch_info(self):
        """(workgroups resident at once, dynamic LDS bytes per workgroup) of the
        persistent launch at the current workgroup size."""
        r, l = _i32(), _i64()
        _check(_lib.gko_batch_launch_info(self.handle, ctypes.byref(r), ctypes.byref(l)))
        return r.value, l.value

    def _outs(self):
        torch = _torch()
        dev = torch.device("cuda", self.ctx.device)
        return (torch.empty(self.nsys, dtype=torch.int32, device=dev),
                torch.empty(self.nsys, dtype=torch.float64, device=dev))

    def solve(self, b, x, tol: float = 1e-10, maxit: int = 1000):
        """Returns (status, iters[nsys] device tensor, relres[nsys] device tensor)."""
        it, rr = self._outs()
        st = _lib.gko_batch_cg_solve(self.handle, _ptr(b), _ptr(x), tol, maxit, _ptr(it), _ptr(rr))
        if st not in (OK, ERR_NOT_CONVERGED, ERR_BREAKDOWN, ERR_NOT_SPD):
            raise GkoError(st, last_error())
        return st, it, rr

    @property
    def lds_mode(self) -> str:
        """"all" (x, r, p, q in LDS) or "direction" (only p; rows and the rest in registers)."""
        m = _i32()
        _check(_lib.gko_batch_get_lds_mode(self.handle, ctypes.byref(m)))
        return BATCH_LDS_MODES[m.value]

    @lds_mode.setter
    def lds_mode(self, mode: str):
        _check(_lib.gko_batch_set_lds_mode(self.handle, BATCH_LDS_MODES.index(mode)))

    def autotune(self, b, x, tol: float = 1e-10, maxit: int = 1000):
        """Times every workgroup size and LDS mode, keeps the fastest pair.
        Returns (block, {(block, mode): ms}) (ms infinite where a mode does not fit)."""
        it, rr = self._outs()
        blk = _i32()
        ms = (ctypes.c_float * (4 * len(BATCH_LDS_MODES)))()
        _check(_lib.gko_batch_autotune(self.handle, _ptr(b), _ptr(x), tol, maxit, _ptr(it),
                                       _ptr(rr), ctypes.byref(blk), ms))
        keys = [(bk, md) for bk in (64, 128, 256, 512) for md in BATCH_LDS_MODES]
        return blk.value, dict(zip(keys, list(ms)))

    def close(self):
        if getattr(self, "handle", None):
            _lib.gko_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------- selector
N_FEATURES = 32
SELECTOR_FORMATS = ("csr", "csr_merge", "coo", "ell", "hybrid", "sellp")   # output order
N_CLASSES = len(SELECTOR_FORMATS)
N_PARAMS = 64 * 32 + 64 + 64 * 64 + 64 + N_CLASSES * 64 + N_CLASSES   # 6662


def _fbuf(n):
    return (ctypes.c_float * n)()


def features(A: Matrix) -> np.ndarray:
    """The 32 structural features of A (float32, host)."""
    f = _fbuf(N_FEATURES)
    _check(_lib.gko_matrix_features(A.handle, f))
    return np.frombuffer(f, dtype=np.float32).copy()


def autotune_format(A: Matrix):
    """Time every format on clones of A.  Returns (best name, float32[6] ms; inf = infeasible)."""
    best = _st()
    ms = _fbuf(N_CLASSES)
    _check(_lib.gko_autotune_format(A.handle, ctypes.byref(best), ms))
    return FORMAT_NAMES[best.value], np.frombuffer(ms, dtype=np.float32).copy()


class Mlp:
    """The selector network (32 -> 64 -> 64 -> 6), parameters and Adam state on the GPU."""

    def __init__(self, params=None, ctx: Context | None = None, handle=None):
        self.ctx = ctx or default_context()
        if handle is not None:
            self.handle = handle
            return
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != N_PARAMS:
            raise ValueError("expected %d parameters" % N_PARAMS)
        h = _vp()
        _check(_lib.gko_mlp_create(self.ctx.handle, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   ctypes.byref(h)))
        self.handle = h

    @classmethod
    def load(cls, path: str, ctx: Context | None = None) -> "Mlp":
        ctx = ctx or default_context()
        h = _vp()
        _check(_lib.gko_mlp_load(ctx.handle, path.encode(), ctypes.byref(h)))
        return cls(ctx=ctx, handle=h)

    def save(self, path: str):
        _check(_lib.gko_mlp_save(self.handle, path.encode()))

    def params(self):
        p, n = _fbuf(N_PARAMS), _fbuf(2 * N_FEATURES)
        _check(_lib.gko_mlp_get_params(self.handle, p, n))
        return (np.frombuffer(p, dtype=np.float32).copy(),
                np.frombuffer(n, dtype=np.float32).copy().reshape(2, N_FEATURES))

    def fit_normalization(self, X):
        _check(_lib.gko_mlp_fit_normalization(self.handle, X.shape[0], _ptr(X)))

    def forward(self, X):
        torch = _torch()
        out = torch.empty((X.shape[0], N_CLASSES), dtype=torch.float32, device=X.device)
        _check(_lib.gko_mlp_forward(self.handle, X.shape[0], _ptr(X), _ptr(out)))
        return out

    def loss_grad(self, X, Y, M):
        torch = _torch()
        g = torch.empty(N_PARAMS, dtype=torch.float32, device=X.device)
        loss = torch.empty((), dtype=torch.float64, device=X.device)
        _check(_lib.gko_mlp_loss_grad(self.handle, X.shape[0], _ptr(X), _ptr(Y), _ptr(M), _ptr(g),
                                      _ptr(loss)))
        return loss, g

    def train(self, X, Y, M, steps: int, lr: float = 1e-3):
        """Full-batch Adam steps on the GPU; returns the loss before each step (device)."""
        torch = _torch()
        hist = torch.empty(steps, dtype=torch.float32, device=X.device)
        _check(_lib.gko_mlp_train(self.handle, X.shape[0], _ptr(X), _ptr(Y), _ptr(M), steps, lr,
                                  _ptr(hist)))
        return hist

    def select(self, A: Matrix):
        """(format name, float32[6] scores) predicted for A."""
        f = _st()
        sc = _fbuf(N_CLASSES)
        _check(_lib.gko_select_format(A.handle, self.handle, ctypes.byref(f), sc))
        return FORMAT_NAMES[f.value], np.frombuffer(sc, dtype=np.float32).copy()

    def close(self):
        if getattr(self, "handle", None):
            _lib.gko_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def set_selector(model: Mlp | None, ctx: Context | None = None):
    """Make gko_convert(A, 'auto') on this context ask model (None: time every format)."""
    ctx = ctx or default_context()
    _check(_lib.gko_context_set_selector(ctx.handle, None if model is None else model.handle))
