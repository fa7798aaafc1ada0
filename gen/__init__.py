"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

Holds none of the method's arithmetic: random draws and sparsity layout only
(see gen.c for the generator definitions).  Matrices come back as host CSR
triples ``(row_ptr int32[n+1], col int32[nnz], val float64[nnz])`` with
columns sorted ascending inside each row.

The workloads mirror the paper's test sets in shape: SpMV over a range of
regular and irregular sparse matrices (Sec. 6.1) and Krylov solves on SPD
problems (Sec. 6.2).  The paper's own matrices are a public collection that is
not available here, so seeded synthetic matrices of the stated shapes stand
in for them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libgen.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile gen.c into libgen.so with gcc (host only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, i64, i32, f64 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    lib.gen_splitmix64_first.argtypes = [u64, ctypes.c_uint]
    lib.gen_splitmix64_first.restype = u64
    lib.gen_uniform.argtypes = [u64, i64, f64, f64, _f64p]
    lib.gen_grid_nnz.argtypes = [i64, i64, i64, ctypes.c_int]
    lib.gen_grid_nnz.restype = i64
    lib.gen_grid_fill.argtypes = [i64, i64, i64, ctypes.c_int, _i32p, _i32p, _f64p]
    lib.gen_convdiff2d_fill.argtypes = [i64, f64, _i32p, _i32p, _f64p]
    lib.gen_lognormal_lengths.argtypes = [u64, i64, f64, f64, i32, i32, ctypes.c_int, _i32p]
    lib.gen_lognormal_lengths.restype = i64
    lib.gen_uniform_lengths.argtypes = [u64, i64, i32, i32, _i32p]
    lib.gen_uniform_lengths.restype = i64
    lib.gen_random_rows_fill.argtypes = [u64, i64, i64, _i32p, _i32p, _i32p, _f64p]
    lib.gen_random_rows_fill.restype = ctypes.c_int
    lib.gen_banded_rows_fill.argtypes = [u64, i64, i64, _i32p, _i32p, _i32p, _f64p]
    lib.gen_banded_rows_fill.restype = ctypes.c_int
    lib.gen_blockdiag.argtypes = [u64, i64, i32, i32, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]
    lib.gen_blockdiag.restype = i64
    lib.gen_batch_dims.argtypes = [u64, i64, i32, i32, _i32p, _i64p, _i32p, _f64p]
    lib.gen_batch_fill.argtypes = [u64, i64, i32, i32, _i64p, _i64p, _i32p, _i32p, _f64p, _f64p]
    _lib = lib
    return lib


def splitmix64_first(seed: int, k: int = 0) -> int:
    """First SplitMix64 output of stream (seed, k) (for pinning the generator)."""
    return int(_load().gen_splitmix64_first(seed, k))


def uniform(seed: int, n: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """n draws of U[lo, hi] from stream (seed, 0)."""
    out = np.empty(n, dtype=np.float64)
    _load().gen_uniform(seed, n, lo, hi, out)
    return out


def grid(nx: int, ny: int = 1, nz: int = 1, kind: str = "star"):
    """Laplacian-type stencil on an nx*ny*nz grid with Dirichlet boundary.

    kind 'star': 3/5/7-point (diagonal 2d), 'box': 9/27-point (diagonal 3^d-1),
    off-diagonals -1.  The 27-point matrix equals 27 I - T(x)T(x)T with T =
    tridiag(1,1,1), the 7-point one is the standard 3D Poisson matrix.
    """
    k = {"star": 0, "box": 1}[kind]
    lib = _load()
    nnz = lib.gen_grid_nnz(nx, ny, nz, k)
    n = nx * ny * nz
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    lib.gen_grid_fill(nx, ny, nz, k, rp, col, val)
    return rp, col, val


def laplace1d(N: int):
    return grid(N)


def laplace2d(N: int):
    return grid(N, N)


def laplace3d(N: int):
    return grid(N, N, N)


def stencil27(N: int):
    return grid(N, N, N, kind="box")


def convdiff2d(N: int, c: float = 0.5):
    """Nonsymmetric 2D convection-diffusion 5-point matrix on an N x N grid."""
    n = N * N
    nnz = 5 * n - 4 * N
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    _load().gen_convdiff2d_fill(N, c, rp, col, val)
    return rp, col, val


def lognormal_lengths(seed: int, n: int, mean: float = 16.0, sigma: float = 1.56,
                      min_len: int = 1, max_len: int = 10000, force_max: bool = True):
    """Row lengths clamp(round(exp(mu + sigma z)), min_len, max_len), mu = ln(mean) - sigma^2/2."""
    mu = math.log(mean) - sigma * sigma / 2.0
    lens = np.empty(n, dtype=np.int32)
    _load().gen_lognormal_lengths(seed, n, mu, sigma, min_len, max_len, int(force_max), lens)
    return lens


def random_rows(seed: int, lens: np.ndarray, n_cols: int):
    """CSR with row i holding lens[i] distinct uniform columns in [0, n_cols), values U[-1,1]."""
    lens = np.ascontiguousarray(lens, dtype=np.int32)
    n = lens.shape[0]
    nnz = int(lens.sum(dtype=np.int64))
    if nnz >= 2**31:
        raise ValueError("nnz exceeds int32 offsets")
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    rc = _load().gen_random_rows_fill(seed, n, n_cols, lens, rp, col, val)
    if rc:
        raise ValueError("random_rows: bad lengths (rc=%d)" % rc)
    return rp, col, val


def random_lognormal(seed: int, n: int, mean: float = 16.0, sigma: float = 1.56,
                     max_len: int = 10000, n_cols: int | None = None):
    """The irregular SpMV workload: lognormal row lengths, uniform distinct columns."""
    lens = lognormal_lengths(seed, n, mean, sigma, 1, max_len, True)
    return random_rows(seed, lens, n if n_cols is None else n_cols)


def uniform_random(seed: int, n: int, lo: int, hi: int, n_cols: int | None = None):
    """Row lengths U{lo..hi}, uniform distinct columns."""
    lens = np.empty(n, dtype=np.int32)
    _load().gen_uniform_lengths(seed, n, lo, hi, lens)
    return random_rows(seed, lens, n if n_cols is None else n_cols)


def banded(seed: int, n: int, bw: int, lo: int, hi: int):
    """Random fill inside the band |i-j| <= bw, row lengths U{lo..hi} clipped to the window."""
    lens = np.empty(n, dtype=np.int32)
    _load().gen_uniform_lengths(seed, n, lo, hi, lens)
    i = np.arange(n, dtype=np.int64)
    window = np.minimum(i + bw, n - 1) - np.maximum(i - bw, 0) + 1
    lens = np.clip(lens, 1, window).astype(np.int32)
    nnz = int(lens.sum(dtype=np.int64))
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    rc = _load().gen_banded_rows_fill(seed, n, bw, lens, rp, col, val)
    if rc:
        raise ValueError("banded: rc=%d" % rc)
    return rp, col, val


def blockdiag(seed: int, n: int, bmin: int, bmax: int):
    """Dense diagonal blocks of sizes U{bmin..bmax}, values U[-1,1]."""
    lib = _load()
    nnz = lib.gen_blockdiag(seed, n, bmin, bmax, None, None, None)
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    lib.gen_blockdiag(seed, n, bmin, bmax, rp.ctypes.data, col.ctypes.data, val.ctypes.data)
    return rp, col, val


@dataclass
class BatchSystems:
    """Concatenated small SPD systems with local CSR indices."""
    m: np.ndarray            # int32[nsys] rows per system
    pattern: np.ndarray      # int32[nsys] 3 or 5
    shift: np.ndarray        # float64[nsys] diagonal shift s
    row_off: np.ndarray      # int64[nsys+1] first row of each system
    nnz_off: np.ndarray      # int64[nsys+1] first entry of each system
    row_ptr: np.ndarray      # int32[row_off[-1] + nsys] local offsets, m_i+1 per system
    col: np.ndarray          # int32[nnz] local column indices
    val: np.ndarray          # float64[nnz]
    xstar: np.ndarray        # float64[row_off[-1]] manufactured solutions

    @property
    def nsys(self) -> int:
        return int(self.m.shape[0])

    def system(self, i: int):
        """Local CSR triple of system i."""
        r0 = int(self.row_off[i]) + i
        m = int(self.m[i])
        k0, k1 = int(self.nnz_off[i]), int(self.nnz_off[i + 1])
        return self.row_ptr[r0:r0 + m + 1], self.col[k0:k1], self.val[k0:k1]


def batch_systems(nsys: int, master_seed: int = 6, m_lo: int = 32, m_hi: int = 1024) -> BatchSystems:
    """nsys SPD systems: sizes U{m_lo..m_hi}, 3- or 5-point pattern, diagonal shift U[0.1, 2]."""
    lib = _load()
    m = np.empty(nsys, dtype=np.int32)
    nnz = np.empty(nsys, dtype=np.int64)
    pat = np.empty(nsys, dtype=np.int32)
    shift = np.empty(nsys, dtype=np.float64)
    lib.gen_batch_dims(master_seed, nsys, m_lo, m_hi, m, nnz, pat, shift)
    row_off = np.zeros(nsys + 1, dtype=np.int64)
    row_off[1:] = np.cumsum(m, dtype=np.int64)
    nnz_off = np.zeros(nsys + 1, dtype=np.int64)
    nnz_off[1:] = np.cumsum(nnz)
    rp = np.empty(int(row_off[-1]) + nsys, dtype=np.int32)
    col = np.empty(int(nnz_off[-1]), dtype=np.int32)
    val = np.empty(int(nnz_off[-1]), dtype=np.float64)
    xs = np.empty(int(row_off[-1]), dtype=np.float64)
    lib.gen_batch_fill(master_seed, nsys, m_lo, m_hi, row_off, nnz_off, rp, col, val, xs)
    return BatchSystems(m, pat, shift, row_off, nnz_off, rp, col, val, xs)


# --------------------------------------------------------------------------- selector corpus
CORPUS_FAMILIES = ("banded", "stencil", "uniform", "powerlaw", "blockdiag")


def corpus_spec(i: int, seed: int = 7, n_lo: float = 1e4, n_hi: float = 1e6) -> dict:
    """Recipe of corpus matrix i: family i mod 5; n log-uniform in [n_lo, n_hi];
    target mean row length U[4, 64]; family parameters from stream (seed*2^20 + i, 0)."""
    u = uniform((seed << 20) + i, 6, 0.0, 1.0)
    fam = CORPUS_FAMILIES[i % 5]
    n = int(round(10 ** (math.log10(n_lo) + (math.log10(n_hi) - math.log10(n_lo)) * u[0])))
    mean = 4.0 + 60.0 * u[1]
    spec = {"index": i, "family": fam, "n": n, "mean": mean, "seed": (seed << 20) + i}
    if fam == "banded":
        spec["bandwidth"] = 1 + int(u[2] * 64)
    elif fam == "stencil":
        spec["stencil"] = ("2d5", "2d9", "3d7", "3d27")[int(u[2] * 4) % 4]
    elif fam == "powerlaw":
        spec["sigma"] = 0.5 + 1.5 * u[3]
    return spec


def corpus_matrix(spec: dict):
    """CSR triple of a corpus recipe."""
    fam, n, mean, s = spec["family"], spec["n"], spec["mean"], spec["seed"]
    lo, hi = max(1, int(mean / 2)), max(1, int(1.5 * mean))
    if fam == "banded":
        return banded(s, n, spec["bandwidth"], lo, hi)
    if fam == "stencil":
        kind = spec["stencil"]
        if kind.startswith("2d"):
            N = max(2, int(round(math.sqrt(n))))
            return grid(N, N, kind="star" if kind == "2d5" else "box")
        N = max(2, int(round(n ** (1.0 / 3.0))))
        return grid(N, N, N, kind="star" if kind == "3d7" else "box")
    if fam == "uniform":
        return uniform_random(s, n, lo, hi)
    if fam == "powerlaw":
        return random_lognormal(s, n, mean=mean, sigma=spec["sigma"], max_len=min(n, 10000))
    if fam == "blockdiag":
        return blockdiag(s, n, 4, 64)
    raise ValueError(fam)
