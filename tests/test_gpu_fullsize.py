"""Parity at the full sizes the bench times, in the same launch configurations.

* SpMV sweep: the 27-point stencil on 128^3 (n = 2,097,152, nnz = 55,742,968) and
  the lognormal random matrix (n = 10^6, longest row 10,000), every format the
  bench runs; all rows are checked against the oracle (the serial C oracle
  handles these sizes in well under a second per SpMV).
* Solvers: block-Jacobi PCG on the 3D 7-point Poisson 256^3 in FP64 and mixed
  precision, in the format the library's AUTO choice picks, checked by the
  oracle's true residual and the manufactured-solution error bound.
* Batched CG: the 10,000-system batch, FP64 and FP32 storage, per-system true
  residuals from the oracle.
"""
import math

import numpy as np
import pytest

from gpu_util import assert_spmv_close, dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


@pytest.fixture(scope="module")
def sweep(gen_mod):
    return {"stencil27_128": gen_mod.stencil27(128),
            "lognormal_1M": gen_mod.random_lognormal(4, 1_000_000, mean=16.0, sigma=1.56,
                                                     max_len=10000)}


@pytest.mark.parametrize("name,fmt", [("stencil27_128", f) for f in
                                      ("csr", "csr_merge", "coo", "ell", "hybrid", "sellp")] +
                         [("lognormal_1M", f) for f in ("csr", "csr_merge", "coo", "hybrid")])
def test_sweep_spmv_full_size(g, orc, gen_mod, sweep, name, fmt):
    import torch
    A = sweep[name]
    n = len(A[0]) - 1
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = gen_mod.uniform(3 if name.startswith("st") else 5, n)
    y = torch.empty(n, dtype=torch.float64, device="cuda")
    g.spmv(M, 1.0, dev(x), 0.0, y)
    ref = orc.spmv_dot2(A, x)
    absy = orc.spmv_absbound(A, x)
    assert_spmv_close(host(y), ref, absy, np.diff(A[0]), False, "%s/%s" % (name, fmt))
    M.close()


@pytest.mark.parametrize("fmt", ["ell", "sellp"])
def test_lognormal_padded_formats_refused(g, sweep, fmt):
    """Independent lognormal row lengths: ELL pads to 88x and unsorted SELL-P
    slices to 15x the nonzeros, both above the 4x storage limit."""
    M = g.Matrix.from_csr(*sweep["lognormal_1M"])
    with pytest.raises(g.GkoError) as e:
        M.convert(fmt)
    assert e.value.status == g.ERR_UNSUPPORTED and M.describe().format == "csr"


@pytest.fixture(scope="module")
def poisson(gen_mod, orc):
    N = 256
    A = gen_mod.laplace3d(N)
    xs = gen_mod.uniform(5, N ** 3)
    b = orc.spmv(A, xs)
    return A, xs, b


@pytest.mark.parametrize("fmt", ["csr", "ell", "sellp"])
def test_poisson256_spmv_full_size(g, orc, gen_mod, poisson, fmt):
    """SpMV on the 7-point Poisson 256^3 (16.8M rows): above the row count up
    to which the row-blocked kernels order their workgroups by XCD, so this
    covers their hardware-order path against the Dot2 oracle."""
    import torch
    A, xs, _ = poisson
    n = len(A[0]) - 1
    M = g.Matrix.from_csr(*A).convert(fmt)
    y = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    g.spmv(M, 1.0, dev(xs), 0.0, y)
    ref = orc.spmv_dot2(A, xs)
    absy = orc.spmv_absbound(A, xs)
    assert_spmv_close(host(y), ref, absy, np.diff(A[0]), False, "poisson256/%s" % fmt)
    M.close()


@pytest.fixture(scope="module")
def poisson_oracle_x(orc, poisson):
    """The oracle's FP64 block-Jacobi(8) PCG solution of the config-3 system
    (serial; about 100 s on one host core)."""
    A, xs, b = poisson
    rc, inv = orc.bj_invert(A, 8)
    rc, x, info = orc.cg(A, b, tol=1e-10, maxit=20000, bj_inv=inv)
    assert rc == orc.OK and info["iters"] == 649, info
    return x


@pytest.mark.timeout(900)
@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_poisson256_pcg_full_size(g, orc, poisson, poisson_oracle_x, mixed):
    """FP64 and mixed-precision PCG at the bench's size: the oracle's true
    residual, the manufactured-solution bound, and the per-solve error
    against the FP64 oracle's own solution within 2 kappa tol."""
    A, xs, b = poisson
    N = 256
    ctx = g.default_context()
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR if mixed else g.PREC_FP64,
                        precond=g.PRECOND_BLOCK_JACOBI, block_size=8, inner_tol=1e-5)
    try:
        M = g.Matrix.from_csr(*A)
        M.convert("auto")
        x = dev(np.zeros(N ** 3))
        info = g.cg(M, dev(b), x, tol=1e-10, maxit=20000)
        assert info["status"] == g.OK, info
        xg = host(x)
        true = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
        assert true <= 1e-10
        kappa = (6 + 6 * math.cos(math.pi / (N + 1))) / (6 - 6 * math.cos(math.pi / (N + 1)))
        assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= kappa * true
        xo = poisson_oracle_x
        assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10
        if not mixed:   # the oracle's recurrence in the same precision: 649 iterations
            assert abs(info["iterations"] - 649) <= 2, info
    finally:
        ctx.set_solver_opts()


@pytest.mark.parametrize("solver", ["fcg", "pipecg"])
def test_poisson256_cg_variants_full_size(g, orc, poisson, solver):
    """Flexible and pipelined block-Jacobi CG at the bench's size, in the
    format AUTO picks: true residual from the oracle's SpMV, error bound."""
    A, xs, b = poisson
    N = 256
    ctx = g.default_context()
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    try:
        M = g.Matrix.from_csr(*A)
        M.convert("auto")
        x = dev(np.zeros(N ** 3))
        info = getattr(g, solver)(M, dev(b), x, tol=1e-10, maxit=20000)
        assert info["status"] == g.OK, info
        assert 600 <= info["iterations"] <= 700, info      # block-Jacobi CG: 649
        xg = host(x)
        true = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
        assert true <= 1e-10
        kappa = (6 + 6 * math.cos(math.pi / (N + 1))) / (6 - 6 * math.cos(math.pi / (N + 1)))
        assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= kappa * true
    finally:
        ctx.set_solver_opts()


def test_poisson256_gmres_estimate_full_size(g, orc, poisson):
    """Two GMRES(30) cycles at the bench's size: the Givens residual estimate
    of the returned iterate equals its true residual (the oracle's SpMV), and
    the cycles reduce it."""
    A, xs, b = poisson
    ctx = g.default_context()
    ctx.set_solver_opts(krylov_dim=30)
    try:
        M = g.Matrix.from_csr(*A)
        M.convert("auto")
        x = dev(np.zeros(256 ** 3))
        info = g.gmres(M, dev(b), x, tol=1e-30, maxit=60)
        assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 60
        true = np.linalg.norm(b - orc.spmv(A, host(x))) / np.linalg.norm(b)
        assert abs(info["rel_residual"] - true) <= 1e-8 * true
        assert abs(info["true_rel_residual"] - true) <= 1e-12
        assert true < 0.2
    finally:
        ctx.set_solver_opts()


@pytest.mark.parametrize("fmt", ["csr", "ell", "sellp"])
@pytest.mark.parametrize("solver", ["bicgstab", "cgs"])
def test_poisson256_nonsymmetric_fused_full_size(g, orc, poisson, solver, fmt):
    """BiCGSTAB and CGS for 20 iterations at the bench's size in each format
    whose SpMV fuses the step's dot products (a 65536-block grid with two
    sums per block for BiCGSTAB's t.s, t.t): the reported true residual is
    the oracle's, and the recurrence's estimate has not drifted from it."""
    A, xs, b = poisson
    M = g.Matrix.from_csr(*A)
    try:
        M.convert(fmt)
        x = dev(np.zeros(256 ** 3))
        info = getattr(g, solver)(M, dev(b), x, tol=1e-30, maxit=20)
        assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 20, info
        true = np.linalg.norm(b - orc.spmv(A, host(x))) / np.linalg.norm(b)
        assert abs(info["true_rel_residual"] - true) <= 1e-12
        assert abs(info["rel_residual"] - true) <= 1e-6 * true
        assert true < 1e-3    # the oracle's 20 iterations: 9.6e-5 (BiCGSTAB), 4.5e-5 (CGS)
    finally:
        M.close()


@pytest.fixture(scope="module")
def laplace1d_big(gen_mod):
    n = (1 << 24) + 4096      # more rows than the fused products' largest grid
    return gen_mod.laplace1d(n), gen_mod.uniform(12, n)


@pytest.mark.parametrize("solver", ["cg", "bicgstab", "cgs"])
def test_sellp_fused_grid_stride(g, orc, laplace1d_big, solver):
    """SELL-P with more than 65536 x 256 rows: the fused products take their
    grid-stride form.  Ten iterations against the oracle's ten."""
    A, b = laplace1d_big
    M = g.Matrix.from_csr(*A)
    try:
        M.convert("sellp")
        x = dev(np.zeros(len(b)))
        info = getattr(g, solver)(M, dev(b), x, tol=1e-30, maxit=10)
        rc, xo, oi = getattr(orc, solver)(A, b, tol=1e-30, maxit=10)
        assert rc == orc.NOT_CONVERGED and oi["iters"] == 10
        assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 10, info
        xg = host(x)
        assert np.abs(xg - xo).max() <= 1e-9 * np.abs(xo).max()
        assert abs(info["rel_residual"] - oi["relres"]) <= 1e-9 * oi["relres"]
    finally:
        M.close()


@pytest.mark.parametrize("f32", [False, True], ids=["fp64", "fp32"])
def test_batch_10k_full_size(g, orc, gen_mod, f32):
    import torch
    B = gen_mod.batch_systems(10000, master_seed=6)
    vals = B.val.astype(np.float32).astype(np.float64) if f32 else B.val
    b = np.empty_like(B.xstar)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        k0, k1 = int(B.nnz_off[i]), int(B.nnz_off[i + 1])
        b[r0:r1] = orc.spmv((B.system(i)[0], B.system(i)[1], vals[k0:k1]), B.xstar[r0:r1])
    G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col,
                B.val.astype(np.float32) if f32 else B.val,
                dtype=torch.float32 if f32 else torch.float64)
    x = dev(np.zeros(B.xstar.shape))
    blk, _ = G.autotune(dev(b), x)
    st, it, rr = G.solve(dev(b), x, tol=1e-10)
    assert st == g.OK
    xg = host(x)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        k0, k1 = int(B.nnz_off[i]), int(B.nnz_off[i + 1])
        r = b[r0:r1] - orc.spmv((B.system(i)[0], B.system(i)[1], vals[k0:k1]), xg[r0:r1])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(b[r0:r1]), i
    if not f32:
        rc, xo, it_o, rr_o = orc.batch_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, b, tol=1e-10)
        assert np.all(np.abs(host(it) - it_o) <= 2)
