"""GPU parity of the Krylov solvers (Sec. 6.2: memory-bound Krylov solvers on
top of SpMV) against the oracle: CG and PCG with block-Jacobi, BiCGSTAB,
mixed-precision iterative refinement, dot/norm, and the failure statuses."""
import math

import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


@pytest.fixture()
def ctx(g):
    c = g.default_context()
    c.set_solver_opts()      # defaults: FP64, no preconditioner
    yield c
    c.set_solver_opts()


def kappa_laplace2d(N):
    return (4 + 4 * math.cos(math.pi / (N + 1))) / (4 - 4 * math.cos(math.pi / (N + 1)))


@pytest.mark.parametrize("fmt,single", [("csr", 1), ("csr", 0), ("csr_merge", 1), ("coo", 1),
                                        ("ell", 1), ("hybrid", 1), ("sellp", 1)])
def test_cg_config1_matches_oracle(g, orc, gen_mod, ctx, fmt, single):
    """single = 1: CSR systems this small run on one workgroup in one launch;
    single = 0 and the other formats: the multi-kernel path."""
    N = 64
    A = gen_mod.laplace2d(N)
    xs = gen_mod.uniform(2, N * N)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.cg(A, b, tol=1e-10)
    ctx.set_solver_opts(single_workgroup=single)
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = dev(np.zeros(N * N))
    info = g.cg(M, dev(b), x, tol=1e-10, maxit=5000)
    assert info["status"] == g.OK, info
    xg = host(x)
    # same recurrence, different rounding: the stop test may trip one step apart
    assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    true = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
    assert true <= 1e-10
    kappa = kappa_laplace2d(N)
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= kappa * true
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10


def kappa_stencil27(N):
    """27-point stencil, 26 on the diagonal and -1 to each neighbour: A = 27 I -
    T x T x T with T = tridiag(1, 1, 1), whose eigenvalues are 1 + 2 cos(k pi/(N+1))."""
    t = 1 + 2 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    prods = np.multiply.outer(np.multiply.outer(t, t), t)
    return (27 - prods.min()) / (27 - prods.max())


def test_cg_csr_four_lanes_per_row_matches_oracle(g, orc, gen_mod, ctx):
    """CG's fused product on the LDS-staged CSR kernel with four lanes per row
    (mean row length >= 12), 9261 rows (a ragged last tile of 64 rows)."""
    N = 21
    A = gen_mod.stencil27(N)
    n = N ** 3
    xs = gen_mod.uniform(3, n)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.cg(A, b, tol=1e-10)
    ctx.set_solver_opts(single_workgroup=0)
    M = g.Matrix.from_csr(*A)
    d = M.describe()
    assert d.csr_kernel == 0 and d.csr_row_lanes == 4, d
    x = dev(np.zeros(n))
    info = g.cg(M, dev(b), x, tol=1e-10, maxit=5000)
    assert info["status"] == g.OK, info
    assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    xg = host(x)
    true = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
    assert true <= 1e-10
    kappa = kappa_stencil27(N)
    assert 60 < kappa < 70
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10


def test_cg_check_every_does_not_change_iterates(g, orc, gen_mod, ctx):
    A = gen_mod.laplace2d(32)
    b = orc.spmv(A, gen_mod.uniform(2, 1024))
    M = g.Matrix.from_csr(*A)
    outs = []
    for ce in (1, 7, 50):
        ctx.set_solver_opts(check_every=ce, single_workgroup=0)
        x = dev(np.zeros(1024))
        info = g.cg(M, dev(b), x, tol=1e-10)
        outs.append((info["iterations"], host(x).view(np.int64)))
    assert outs[0][0] == outs[1][0] == outs[2][0]
    assert np.array_equal(outs[0][1], outs[1][1]) and np.array_equal(outs[0][1], outs[2][1])


def test_pcg_block_jacobi_matches_oracle(g, orc, gen_mod, ctx):
    N = 24
    A = gen_mod.laplace3d(N)
    n = N ** 3
    xs = gen_mod.uniform(5, n)
    b = orc.spmv(A, xs)
    rc, inv = orc.bj_invert(A, 8)
    rc, xo, info_o = orc.cg(A, b, tol=1e-10, bj_inv=inv)
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    M = g.Matrix.from_csr(*A)
    x = dev(np.zeros(n))
    info = g.cg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK
    assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    xg = host(x)
    assert np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b) <= 1e-10


def test_pcg_exact_block_preconditioner_one_iteration(g, orc, ctx):
    rng = np.random.default_rng(9)
    n, bs = 64, 8
    rp, col, val = [0], [], []
    for b0 in range(0, n, bs):
        G = rng.standard_normal((bs, bs))
        B = G @ G.T + bs * np.eye(bs)
        for i in range(bs):
            col += list(range(b0, b0 + bs))
            val += list(B[i])
            rp.append(len(col))
    A = (np.array(rp, np.int32), np.array(col, np.int32), np.array(val))
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=bs)
    M = g.Matrix.from_csr(*A)
    bvec = rng.uniform(-1, 1, n)
    x = dev(np.zeros(n))
    info = g.cg(M, dev(bvec), x, tol=1e-12)
    assert info["status"] == g.OK and info["iterations"] == 1


def test_mixed_ir_reaches_fp64_residual(g, orc, gen_mod, ctx):
    N = 32
    A = gen_mod.laplace3d(N)
    n = N ** 3
    xs = gen_mod.uniform(5, n)
    b = orc.spmv(A, xs)
    rc, inv = orc.bj_invert(A, 8)
    rc, x64, _ = orc.cg(A, b, tol=1e-10, bj_inv=inv)
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR, precond=g.PRECOND_BLOCK_JACOBI, block_size=8,
                        inner_tol=1e-5)
    M = g.Matrix.from_csr(*A)
    x = dev(np.zeros(n))
    info = g.cg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK, info
    assert 2 <= info["outer_iterations"] <= 6
    xg = host(x)
    true = np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b)
    assert true <= 1e-10
    kappa = (6 + 6 * math.cos(math.pi / (N + 1))) / (6 - 6 * math.cos(math.pi / (N + 1)))
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    assert np.linalg.norm(xg - x64) / np.linalg.norm(x64) <= 2 * kappa * 1e-10
    # the oracle's mixed solve takes a comparable number of steps, outer and
    # inner: the same recurrences in FP32, so each inner solve's stop test may
    # trip a step or two apart
    rc, xo, info_o = orc.ir_cg(A, b, tol=1e-10, inner_tol=1e-5, bj_inv=inv)
    assert abs(info["outer_iterations"] - info_o["outer_iters"]) <= 1
    slack = 2 * max(info["outer_iterations"], info_o["outer_iters"]) + 2
    assert abs(info["iterations"] - info_o["inner_iters"]) <= slack, (info, info_o)
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10


def test_mixed_ir_maxit_caps_inner_total(g, orc, gen_mod, ctx):
    """With mixed precision, maxit bounds the inner iterations summed over
    the refinement steps, for every CG variant; the oracle stops on the same
    budget."""
    N = 24
    A = gen_mod.laplace3d(N)
    n = N ** 3
    b = orc.spmv(A, gen_mod.uniform(5, n))
    rc, inv = orc.bj_invert(A, 8)
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR, precond=g.PRECOND_BLOCK_JACOBI, block_size=8,
                        inner_tol=1e-5)
    M = g.Matrix.from_csr(*A)
    rc, xo, info_o = orc.ir_cg(A, b, tol=1e-10, inner_tol=1e-5, bj_inv=inv, maxit=30)
    assert rc == orc.NOT_CONVERGED and info_o["inner_iters"] == 30
    for solve in (g.cg, g.fcg, g.pipecg):
        for maxit in (0, 1, 30):
            info = solve(M, dev(b), dev(np.zeros(n)), tol=1e-10, maxit=maxit)
            assert info["status"] == g.ERR_NOT_CONVERGED, (solve.__name__, maxit, info)
            assert info["iterations"] <= maxit, (solve.__name__, maxit, info)
        assert info["iterations"] == 30


def test_solvers_reject_overlapping_b_and_x(g, gen_mod, ctx):
    """b is re-read after x changes, so every solver refuses aliased b and x."""
    A = g.Matrix.from_csr(*gen_mod.laplace2d(16))
    buf = dev(np.ones(512))
    for solve in (g.cg, g.fcg, g.pipecg, g.bicgstab, g.cgs, g.gmres):
        assert solve(A, buf, buf)["status"] == g.ERR_INVALID_ARG, solve.__name__
        assert solve(A, buf[:256], buf[100:356])["status"] == g.ERR_INVALID_ARG
        info = solve(A, buf[:256], buf[256:], tol=1e-8)
        assert info["status"] == g.OK, (solve.__name__, info)


def test_bicgstab_convdiff(g, orc, gen_mod, ctx):
    A = gen_mod.convdiff2d(40, 0.5)
    xs = gen_mod.uniform(8, 1600)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.bicgstab(A, b, tol=1e-10)
    # CSR, ELL, HYB without a tail and SELL-P fuse r̂·v and t·s, t·t into their
    # SpMVs; COO and merge-path run separate dot kernels
    for fmt in ["csr", "csr_merge", "coo", "ell", "hybrid", "sellp"]:
        M = g.Matrix.from_csr(*A).convert(fmt)
        x = dev(np.zeros(1600))
        info = g.bicgstab(M, dev(b), x, tol=1e-10)
        assert info["status"] == g.OK, info
        xg = host(x)
        assert np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b) <= 1.01e-10
        # iteration counts are not pinned for BiCGSTAB; they should still be close
        assert abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 10)


@pytest.mark.parametrize("single", [1, 0])
def test_solver_statuses(g, gen_mod, ctx, single):
    ctx.set_solver_opts(single_workgroup=single)
    A = gen_mod.laplace1d(20)
    M = g.Matrix.from_csr(*A)
    x = dev(np.ones(20))
    info = g.cg(M, dev(np.zeros(20)), x)
    assert info["status"] == g.OK and info["iterations"] == 0 and host(x).max() == 0
    b = np.ones(20)
    b[3] = np.nan
    assert g.cg(M, dev(b), dev(np.zeros(20)))["status"] == g.ERR_BREAKDOWN
    D = g.Matrix.from_csr(np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32),
                          np.array([1.0, 2.0, -1.0, 3.0]))
    assert g.cg(D, dev(np.ones(4)), dev(np.zeros(4)))["status"] == g.ERR_NOT_SPD
    L = g.Matrix.from_csr(*gen_mod.laplace2d(32))
    info = g.cg(L, dev(np.ones(1024)), dev(np.zeros(1024)), tol=1e-10, maxit=5)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 5
    with pytest.raises(g.GkoError):
        g.cg(L, dev(np.ones(1024)), dev(np.zeros(1024)), tol=-1.0, raise_on_failure=True)
    # BiCGSTAB breakdown: rhat.v = 0 at the first step
    B = g.Matrix.from_csr(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.ones(2))
    assert g.bicgstab(B, dev(np.array([1.0, 0.0])), dev(np.zeros(2)))["status"] == g.ERR_BREAKDOWN
    # singular diagonal block
    S = g.Matrix.from_csr(np.array([0, 1, 1, 2], np.int32), np.array([0, 2], np.int32), np.ones(2))
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=4)
    assert g.cg(S, dev(np.ones(3)), dev(np.zeros(3)))["status"] == g.ERR_BREAKDOWN


def test_single_workgroup_cg_size_limits(g, orc, gen_mod, ctx):
    """The largest 2D Laplacian the one-workgroup path takes (90^2 = 8100 rows,
    8 rows per thread) and one just above it (91^2, multi-kernel path) both
    meet the oracle; the two paths agree on the iteration count within the
    rounding slack of the stopping test."""
    for N in (90, 91):
        A = gen_mod.laplace2d(N)
        n = N * N
        b = orc.spmv(A, gen_mod.uniform(2, n))
        rc, xo, info_o = orc.cg(A, b, tol=1e-10)
        M = g.Matrix.from_csr(*A)
        for single in (1, 0):
            ctx.set_solver_opts(single_workgroup=single)
            x = dev(np.zeros(n))
            info = g.cg(M, dev(b), x, tol=1e-10, maxit=5000)
            assert info["status"] == g.OK, (N, single, info)
            assert abs(info["iterations"] - info_o["iters"]) <= 2, (N, single, info, info_o)
            xg = host(x)
            assert np.linalg.norm(b - orc.spmv(A, xg)) / np.linalg.norm(b) <= 1e-10
            assert info["true_rel_residual"] <= 1e-10


def test_single_workgroup_cg_nonzero_guess_and_repeatable(g, orc, gen_mod, ctx):
    """x on entry is the initial guess; two identical solves agree bitwise."""
    A = gen_mod.laplace2d(40)
    n = 1600
    b = orc.spmv(A, gen_mod.uniform(2, n))
    x0 = gen_mod.uniform(11, n)
    rc, xo, info_o = orc.cg(A, b, tol=1e-10, x0=x0)
    M = g.Matrix.from_csr(*A)
    outs = []
    for _ in range(2):
        x = dev(x0.copy())
        info = g.cg(M, dev(b), x, tol=1e-10)
        assert info["status"] == g.OK
        assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
        outs.append(host(x).view(np.int64))
    assert np.array_equal(outs[0], outs[1])


def test_dot_norm(g, orc, gen_mod):
    import torch
    for n in [0, 1, 255, 256, 257, 100000, 3000017]:
        x = gen_mod.uniform(1, n)
        y = gen_mod.uniform(2, n)
        d = float(host(g.dot(dev(x), dev(y))))
        ref = math.fsum(x * y)
        assert abs(d - ref) <= 2 * n * 2.0 ** -53 * float(np.abs(x * y).sum()) + 1e-300
        nr = float(host(g.norm2(dev(x))))
        assert abs(nr - math.sqrt(math.fsum(x * x))) <= (n + 2) * 2.0 ** -53 * max(nr, 1e-300)
        d32 = float(host(g.dot(dev(x, torch.float32), dev(y, torch.float32))))
        x32, y32 = x.astype(np.float32).astype(np.float64), y.astype(np.float32).astype(np.float64)
        assert abs(d32 - math.fsum(x32 * y32)) <= 2 * n * 2.0 ** -53 * float(np.abs(x32 * y32).sum()) + 1e-300
    # bitwise repeatable
    x = dev(gen_mod.uniform(3, 1 << 20))
    r = [float(host(g.dot(x, x))) for _ in range(3)]
    assert r[0] == r[1] == r[2]


def test_stream_probe_exact(g, gen_mod):
    import torch
    n = 1_000_003
    a, b = gen_mod.uniform(1, n), gen_mod.uniform(2, n)
    c = dev(np.full(n, np.nan))
    g.stream(g.STREAM_COPY, dev(a), c)
    assert np.array_equal(host(c), a)
    g.stream(g.STREAM_TRIAD, dev(a), c, dev(b), 0.37)
    # two roundings (no fused multiply-add), exactly as numpy computes it
    assert np.array_equal(host(c).view(np.int64), (a + 0.37 * b).view(np.int64))
    # arrays off the 16-byte grid take the one-element-per-thread kernels
    ad, cd = dev(a), dev(np.full(n, np.nan))
    g.stream(g.STREAM_COPY, ad[1:], cd[1:])
    assert np.array_equal(host(cd)[1:], a[1:]) and np.isnan(host(cd)[0])
    for m in (1, 2, 3):
        c = dev(np.full(m, np.nan))
        g.stream(g.STREAM_COPY, dev(a[:m]), c)
        assert np.array_equal(host(c), a[:m])


def test_gather_probe_exact(g, gen_mod):
    """y = x[idx] bit for bit, including a ragged tail; indices outside x read 0."""
    import torch
    m, n = 1_000_003, 2_000_001
    x = gen_mod.uniform(1, m)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, m, n).astype(np.int32)
    idx[7] = -3
    idx[n - 1] = m
    y = dev(np.full(n, np.nan))
    g.gather_probe(dev(x), dev(idx), y)
    want = np.where((idx >= 0) & (idx < m), x[np.clip(idx, 0, m - 1)], 0.0)
    assert np.array_equal(host(y).view(np.int64), want.view(np.int64))
    with pytest.raises(g.GkoError):
        g.gather_probe(dev(x), dev(idx)[1:], y[1:])     # idx and y off the 16-byte grid


def test_solver_statuses_large_grids(g, gen_mod, ctx):
    """The failure statuses also come out right when the reductions finish in
    the separate finalize kernel (grids of more than 64 blocks)."""
    ctx.set_solver_opts(single_workgroup=0)
    n = 200_000
    L = g.Matrix.from_csr(*gen_mod.laplace2d(448))   # 200,704 rows
    m = L.describe().n_rows
    b = np.ones(m)
    b[12345] = np.nan
    assert g.cg(L, dev(b), dev(np.zeros(m)))["status"] == g.ERR_BREAKDOWN
    info = g.cg(L, dev(np.ones(m)), dev(np.zeros(m)), tol=1e-10, maxit=7)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 7
    d = np.ones(n)
    d[n // 2] = -1.0
    D = g.Matrix.from_csr(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d)
    rhs = np.zeros(n)
    rhs[n // 2] = 1.0
    assert g.cg(D, dev(rhs), dev(np.zeros(n)))["status"] == g.ERR_NOT_SPD
    # BiCGSTAB on the same diagonal converges (it does not need SPD)
    info = g.bicgstab(D, dev(rhs), dev(np.zeros(n)), tol=1e-12)
    assert info["status"] == g.OK, info
    x = dev(np.zeros(m))
    info = g.cg(L, dev(np.ones(m)), x, tol=1e-8)
    assert info["status"] == g.OK and info["true_rel_residual"] <= 1e-8
