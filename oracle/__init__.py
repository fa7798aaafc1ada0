"""ORACLE -- test infrastructure, not part of the product.

Plain serial FP64 CPU implementations (oracle.c, compiled with gcc
``-O2 -ffp-contract=off``) of everything the GPU library computes, used only
by ``tests/``, the smoke check and the bench's CPU-baseline leg.  It shares no
code with the GPU path and never imports it.

Every function takes and returns numpy arrays.  CSR matrices are
``(row_ptr int32[n+1], col int32[nnz], val float64[nnz])`` triples.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, BAD, NOT_CONVERGED, BREAKDOWN, NOT_SPD = 0, 1, 6, 7, 8

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc: no FMA contraction, no fast-math."""
    srcs = [_SRC] + [os.path.join(_HERE, f) for f in sorted(os.listdir(_HERE))
                     if f.endswith(".c") and f != "oracle.c"]
    newest = max(os.path.getmtime(s) for s in srcs)
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared",
                               "-ffp-contract=off", "-fno-fast-math"] + srcs +
                              ["-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    vp = ctypes.c_void_p
    lib.orc_csr_spmv.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, f64, f64, _f64p]
    lib.orc_csr_spmv_absbound.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, f64, f64, _f64p, _f64p]
    lib.orc_csr_spmv_dot2.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, f64, f64, _f64p]
    lib.orc_csr_to_coo.argtypes = [i64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
    lib.orc_max_row_len.argtypes = [i64, _i32p]
    lib.orc_max_row_len.restype = i32
    lib.orc_csr_to_ell.argtypes = [i64, _i32p, _i32p, _f64p, i32, i64, _i32p, _f64p]
    lib.orc_hyb_width.argtypes = [i64, _i32p, i32]
    lib.orc_hyb_width.restype = i32
    lib.orc_hyb_tail_nnz.argtypes = [i64, _i32p, i32]
    lib.orc_hyb_tail_nnz.restype = i64
    lib.orc_csr_to_hyb.argtypes = [i64, _i32p, _i32p, _f64p, i32, i64, _i32p, _f64p,
                                   _i32p, _i32p, _f64p]
    lib.orc_coo_to_csr.argtypes = [i64, i64, _i32p, _i32p, _f64p, _i32p, _i32p, _f64p]
    lib.orc_hyb_to_csr.argtypes = [i64, i32, i64, _i32p, _f64p, i64, _i32p, _i32p, _f64p,
                                   _i32p, _i32p, _f64p]
    lib.orc_sellp_layout.argtypes = [i64, _i32p, i32, _i32p, _i64p]
    lib.orc_sellp_layout.restype = i64
    lib.orc_csr_to_sellp.argtypes = [i64, _i32p, _i32p, _f64p, i32, _i32p, _i64p, _i32p, _f64p]
    lib.orc_sellp_to_csr.argtypes = [i64, i32, _i32p, _i64p, _i32p, _f64p, _i32p, _i32p, _f64p]
    lib.orc_cgs.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32, _f64p]
    lib.orc_gmres.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32, i32, _f64p]
    lib.orc_dot.argtypes = [i64, _f64p, _f64p]
    lib.orc_dot.restype = f64
    lib.orc_norm2.argtypes = [i64, _f64p]
    lib.orc_norm2.restype = f64
    lib.orc_bj_invert.argtypes = [i64, _i32p, _i32p, _f64p, i32, _f64p]
    lib.orc_bj_apply.argtypes = [i64, i32, _f64p, _f64p, _f64p]
    lib.orc_cg.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32, vp, i32, _f64p]
    lib.orc_fcg.argtypes = lib.orc_cg.argtypes
    lib.orc_pipecg.argtypes = lib.orc_cg.argtypes
    lib.orc_bicgstab.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32, _f64p]
    lib.orc_ir_cg.argtypes = [i64, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32, f64, i32, i32,
                              vp, i32, _f64p, _i32p]
    lib.orc_pcg_f32.argtypes = [i64, _i32p, _i32p, _f32p, _f32p, _f32p, f64, i32, vp, i32,
                                ctypes.POINTER(i32)]
    lib.orc_pcg_f32.restype = i32
    lib.orc_bj_apply_f32.argtypes = [i64, i32, _f32p, _f32p, _f32p]
    lib.orc_batch_cg.argtypes = [i64, _i64p, _i64p, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32,
                                 _i32p, _f64p]
    lib.orc_batch_ir_cg.argtypes = [i64, _i64p, _i64p, _i32p, _i32p, _f64p, _f64p, _f64p, f64, i32,
                                    _i32p, _f64p]
    lib.orc_features.argtypes = [i64, i64, _i32p, _i32p, _f64p]
    lib.orc_mlp_forward.argtypes = [i64, _f64p, _f64p, _f64p]
    lib.orc_mlp_loss_grad.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, _f64p]
    lib.orc_mlp_loss_grad.restype = f64
    lib.orc_adam_step.argtypes = [i64, _f64p, _f64p, _f64p, _f64p, i64, f64, f64, f64, f64]
    _lib = lib
    return lib


def _csr(A):
    rp, col, val = A
    return (np.ascontiguousarray(rp, dtype=np.int32), np.ascontiguousarray(col, dtype=np.int32),
            np.ascontiguousarray(val, dtype=np.float64))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------- SpMV
def spmv(A, x, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """y <- alpha A x + beta y, rows summed in ascending storage order."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    out = np.zeros(n) if y is None else _f64(y).copy()
    _load().orc_csr_spmv(n, rp, col, val, _f64(x), alpha, beta, out)
    return out


def spmv_absbound(A, x, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """|alpha| |A| |x| + |beta| |y| per row: the scale of SpMV rounding errors."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    yy = np.zeros(n) if y is None else _f64(y)
    out = np.empty(n)
    _load().orc_csr_spmv_absbound(n, rp, col, val, _f64(x), alpha, beta, yy, out)
    return out


def spmv_dot2(A, x, alpha: float = 1.0, beta: float = 0.0, y=None) -> np.ndarray:
    """SpMV with compensated (Dot2) row sums: error about u^2 |A||x| plus one rounding."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    out = np.zeros(n) if y is None else _f64(y).copy()
    _load().orc_csr_spmv_dot2(n, rp, col, val, _f64(x), alpha, beta, out)
    return out


# --------------------------------------------------------------------------- conversions
def ell_ld(n: int) -> int:
    """ELL leading dimension: n rounded up to a multiple of 64."""
    return (n + 63) // 64 * 64


def csr_to_coo(A):
    rp, col, val = _csr(A)
    n, nnz = rp.shape[0] - 1, col.shape[0]
    r, c, v = np.empty(nnz, np.int32), np.empty(nnz, np.int32), np.empty(nnz, np.float64)
    _load().orc_csr_to_coo(n, rp, col, val, r, c, v)
    return r, c, v


def max_row_len(A) -> int:
    rp = _csr(A)[0]
    return int(_load().orc_max_row_len(rp.shape[0] - 1, rp))


def csr_to_ell(A, K: int | None = None):
    """Column-major padded ELL: returns (K, ld, col[K*ld], val[K*ld])."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    if K is None:
        K = max_row_len(A)
    ld = ell_ld(n)
    ec, ev = np.empty(K * ld, np.int32), np.empty(K * ld, np.float64)
    _load().orc_csr_to_ell(n, rp, col, val, K, ld, ec, ev)
    return K, ld, ec, ev


def hyb_width(A, value_bytes: int = 8) -> int:
    rp = _csr(A)[0]
    return int(_load().orc_hyb_width(rp.shape[0] - 1, rp, value_bytes))


def csr_to_hyb(A, value_bytes: int = 8, K: int | None = None):
    """Returns (K, ld, ell_col, ell_val, tail_row, tail_col, tail_val)."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    lib = _load()
    if K is None:
        K = int(lib.orc_hyb_width(n, rp, value_bytes))
    ld = ell_ld(n)
    t = int(lib.orc_hyb_tail_nnz(n, rp, K))
    ec, ev = np.empty(K * ld, np.int32), np.empty(K * ld, np.float64)
    tr, tc, tv = np.empty(t, np.int32), np.empty(t, np.int32), np.empty(t, np.float64)
    lib.orc_csr_to_hyb(n, rp, col, val, K, ld, ec, ev, tr, tc, tv)
    return K, ld, ec, ev, tr, tc, tv


def coo_to_csr(n: int, row, col, val):
    row, col, val = (np.ascontiguousarray(row, np.int32), np.ascontiguousarray(col, np.int32),
                     _f64(val))
    nnz = row.shape[0]
    rp, c, v = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz, np.float64)
    _load().orc_coo_to_csr(n, nnz, row, col, val, rp, c, v)
    return rp, c, v


def hyb_to_csr(n: int, K: int, ld: int, ecol, evals, trow=None, tcol=None, tval=None):
    """ELL (no tail) or HYB back to CSR, padding dropped."""
    ecol = np.ascontiguousarray(ecol, np.int32)
    evals = _f64(evals)
    if trow is None:
        trow, tcol, tval = (np.empty(0, np.int32), np.empty(0, np.int32), np.empty(0))
    trow, tcol, tval = (np.ascontiguousarray(trow, np.int32), np.ascontiguousarray(tcol, np.int32),
                        _f64(tval))
    nnz = int((ecol >= 0).sum()) + trow.shape[0]
    rp, c, v = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz, np.float64)
    _load().orc_hyb_to_csr(n, K, ld, ecol, evals, trow.shape[0], trow, tcol, tval, rp, c, v)
    return rp, c, v


SELLP_SLICE = 64   # rows per SELL-P slice (one wavefront)


def csr_to_sellp(A, C: int = SELLP_SLICE):
    """SELL-P (sliced ELL, padding per slice): returns (widths, sets, col, val)."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    ns = (n + C - 1) // C
    lib = _load()
    widths, sets = np.empty(ns, np.int32), np.empty(ns + 1, np.int64)
    slots = int(lib.orc_sellp_layout(n, rp, C, widths, sets))
    sc, sv = np.empty(slots, np.int32), np.empty(slots, np.float64)
    lib.orc_csr_to_sellp(n, rp, col, val, C, widths, sets, sc, sv)
    return widths, sets, sc, sv


def sellp_to_csr(n: int, widths, sets, scol, sval, C: int = SELLP_SLICE):
    widths = np.ascontiguousarray(widths, np.int32)
    sets = np.ascontiguousarray(sets, np.int64)
    scol = np.ascontiguousarray(scol, np.int32)
    sval = _f64(sval)
    nnz = int((scol >= 0).sum())
    rp, c, v = np.empty(n + 1, np.int32), np.empty(nnz, np.int32), np.empty(nnz, np.float64)
    _load().orc_sellp_to_csr(n, C, widths, sets, scol, sval, rp, c, v)
    return rp, c, v


# --------------------------------------------------------------------------- BLAS-1
def dot(x, y) -> float:
    x, y = _f64(x), _f64(y)
    return float(_load().orc_dot(x.shape[0], x, y))


def norm2(x) -> float:
    x = _f64(x)
    return float(_load().orc_norm2(x.shape[0], x))


# --------------------------------------------------------------------------- block-Jacobi
def bj_invert(A, bs: int = 8):
    """Explicit inverses of the bs x bs diagonal blocks (Gauss-Jordan, partial pivoting).

    Returns (status, inv[nblocks, bs, bs])."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    nb = (n + bs - 1) // bs
    inv = np.zeros(nb * bs * bs)
    rc = _load().orc_bj_invert(n, rp, col, val, bs, inv)
    return rc, inv.reshape(nb, bs, bs)


def bj_apply(inv, r, bs: int = 8):
    inv = _f64(inv.reshape(-1))
    r = _f64(r)
    z = np.empty_like(r)
    _load().orc_bj_apply(r.shape[0], bs, inv, r, z)
    return z


# --------------------------------------------------------------------------- solvers
def cg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, bj_inv=None, bs: int = 8):
    """(P)CG.  Returns (status, x, info) with info = {iters, relres, true_relres, restarts}."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    inv = None if bj_inv is None else _f64(np.asarray(bj_inv).reshape(-1))
    rc = _load().orc_cg(n, rp, col, val, _f64(b), x, tol, maxit,
                        None if inv is None else inv.ctypes.data, bs, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2],
                   "restarts": int(out[3])}


def bicgstab(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000):
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(3)
    rc = _load().orc_bicgstab(n, rp, col, val, _f64(b), x, tol, maxit, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2]}


def fcg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, bj_inv=None, bs: int = 8):
    """Flexible (P)CG, Polak-Ribiere beta.  Returns (status, x, info) as cg()."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    inv = None if bj_inv is None else _f64(np.asarray(bj_inv).reshape(-1))
    rc = _load().orc_fcg(n, rp, col, val, _f64(b), x, tol, maxit,
                         None if inv is None else inv.ctypes.data, bs, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2],
                   "restarts": int(out[3])}


def pipecg(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, bj_inv=None, bs: int = 8):
    """Pipelined (P)CG (Ghysels-Vanroose).  Returns (status, x, info) as cg()."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    inv = None if bj_inv is None else _f64(np.asarray(bj_inv).reshape(-1))
    rc = _load().orc_pipecg(n, rp, col, val, _f64(b), x, tol, maxit,
                            None if inv is None else inv.ctypes.data, bs, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2],
                   "restarts": int(out[3])}


def cgs(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000):
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(3)
    rc = _load().orc_cgs(n, rp, col, val, _f64(b), x, tol, maxit, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2]}


def gmres(A, b, x0=None, tol: float = 1e-10, maxit: int = 10000, m: int = 30):
    """Restarted GMRES(m).  info = {iters (Arnoldi steps), relres, true_relres, cycles}."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(4)
    rc = _load().orc_gmres(n, rp, col, val, _f64(b), x, tol, maxit, m, out)
    return rc, x, {"iters": int(out[0]), "relres": out[1], "true_relres": out[2],
                   "cycles": int(out[3])}


def ir_cg(A, b, x0=None, tol: float = 1e-10, max_outer: int = 20, inner_tol: float = 1e-5,
          max_inner: int = 1000, bj_inv=None, bs: int = 8, maxit: int = 2 ** 31 - 1):
    """FP64 iterative refinement around an FP32 inner PCG.

    info = {inner_iters (total), outer_iters, true_relres, inner_per_outer (list)}.
    maxit caps the inner iterations summed over the outer steps."""
    rp, col, val = _csr(A)
    n = rp.shape[0] - 1
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    out = np.zeros(3)
    counts = np.zeros(max(max_outer, 1), np.int32)
    inv = None if bj_inv is None else _f64(np.asarray(bj_inv).reshape(-1))
    rc = _load().orc_ir_cg(n, rp, col, val, _f64(b), x, tol, max_outer, inner_tol, max_inner,
                           maxit, None if inv is None else inv.ctypes.data, bs, out, counts)
    outer = int(out[1])
    # an outer step whose inner solve broke down is counted in inner but not in outer
    steps = outer + (1 if rc in (NOT_SPD, BREAKDOWN) else 0)
    return rc, x, {"inner_iters": int(out[0]), "outer_iters": outer,
                   "true_relres": out[2], "inner_per_outer": [int(c) for c in counts[:steps]]}


def pcg_f32(A32, rhs, tol: float, maxit: int = 1000, inv32=None, bs: int = 8):
    """The inner FP32 PCG of ir_cg on its own, from d = 0.

    A32 = (row_ptr, col, float32 values); rhs and inv32 (nblocks*bs*bs, row-major
    blocks) float32.  Returns (status, d float32, iterations)."""
    rp = np.ascontiguousarray(A32[0], np.int32)
    col = np.ascontiguousarray(A32[1], np.int32)
    v32 = np.ascontiguousarray(A32[2], np.float32)
    rhs = np.ascontiguousarray(rhs, np.float32)
    n = rp.shape[0] - 1
    d = np.zeros(n, np.float32)
    inv = None if inv32 is None else np.ascontiguousarray(np.asarray(inv32).reshape(-1), np.float32)
    st = ctypes.c_int32(0)
    it = _load().orc_pcg_f32(n, rp, col, v32, rhs, d, tol, maxit,
                             None if inv is None else inv.ctypes.data, bs, ctypes.byref(st))
    return int(st.value), d, int(it)


def bj_apply_f32(inv32, r32, bs: int = 8):
    """z = D^-1 r blockwise in FP32 arithmetic (the inner solve's preconditioner)."""
    inv = np.ascontiguousarray(np.asarray(inv32).reshape(-1), np.float32)
    r = np.ascontiguousarray(r32, np.float32)
    z = np.empty_like(r)
    _load().orc_bj_apply_f32(r.shape[0], bs, inv, r, z)
    return z


def batch_cg(row_off, nnz_off, rp_local, col, val, b, tol: float = 1e-10, maxit: int = 10000):
    """Per-system CG loop.  Returns (status, x, iters[nsys], true_relres[nsys])."""
    row_off = np.ascontiguousarray(row_off, np.int64)
    nnz_off = np.ascontiguousarray(nnz_off, np.int64)
    nsys = row_off.shape[0] - 1
    x = np.zeros(int(row_off[-1]))
    it = np.zeros(nsys, np.int32)
    rr = np.zeros(nsys)
    rc = _load().orc_batch_cg(nsys, row_off, nnz_off, np.ascontiguousarray(rp_local, np.int32),
                              np.ascontiguousarray(col, np.int32), _f64(val), _f64(b), x, tol,
                              maxit, it, rr)
    return rc, x, it, rr


def batch_ir_cg(row_off, nnz_off, rp_local, col, val, b, tol: float = 1e-10, max_inner: int = 1000):
    """Per-system FP64 refinement around FP32 CG.  Returns (status, x, iters, true_relres)."""
    row_off = np.ascontiguousarray(row_off, np.int64)
    nnz_off = np.ascontiguousarray(nnz_off, np.int64)
    nsys = row_off.shape[0] - 1
    x = np.zeros(int(row_off[-1]))
    it = np.zeros(nsys, np.int32)
    rr = np.zeros(nsys)
    rc = _load().orc_batch_ir_cg(nsys, row_off, nnz_off, np.ascontiguousarray(rp_local, np.int32),
                                 np.ascontiguousarray(col, np.int32), _f64(val), _f64(b), x, tol,
                                 max_inner, it, rr)
    return rc, x, it, rr


# --------------------------------------------------------------------------- selector
N_FEATURES = 32
N_CLASSES = 6      # SpMV formats scored: CSR, CSR merge, COO, ELL, HYB, SELL-P
MLP_SHAPES = [(64, 32), (64,), (64, 64), (64,), (N_CLASSES, 64), (N_CLASSES,)]
N_PARAMS = 6662


def features(A, n_cols: int | None = None) -> np.ndarray:
    """The 32 structural features (FP64), see selector.c for the list."""
    rp, col, _ = _csr(A)
    n = rp.shape[0] - 1
    f = np.zeros(N_FEATURES)
    _load().orc_features(n, n if n_cols is None else n_cols, rp, col, f)
    return f


def mlp_forward(P, X) -> np.ndarray:
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 32)
    out = np.zeros((X.shape[0], N_CLASSES))
    _load().orc_mlp_forward(X.shape[0], _f64(P), X, out)
    return out


def mlp_loss_grad(P, X, Y, M):
    """Masked mean-squared loss and its gradient w.r.t. the 6662 parameters."""
    X = np.ascontiguousarray(X, np.float64).reshape(-1, 32)
    Y = np.ascontiguousarray(Y, np.float64).reshape(-1, N_CLASSES)
    M = np.ascontiguousarray(M, np.float64).reshape(-1, N_CLASSES)
    G = np.zeros(N_PARAMS)
    loss = _load().orc_mlp_loss_grad(X.shape[0], _f64(P), X, Y, M, G)
    return float(loss), G


def adam_step(P, G, m, v, t: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """In place: the t-th Adam update of P, m, v (t >= 1)."""
    _load().orc_adam_step(P.shape[0], P, _f64(G), m, v, t, lr, b1, b2, eps)
