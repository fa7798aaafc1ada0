"""GPU parity of the Krylov solvers beyond CG and BiCGSTAB: flexible CG, CGS
and restarted GMRES, each against its pinned FP64 oracle on the same seeded
inputs (iteration counts within the rounding slack of the stopping tests,
true residuals, manufactured-solution error bounds), in several storage
formats, plus their status paths."""
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
    c.set_solver_opts()
    yield c
    c.set_solver_opts()


def relres(orc, A, b, x):
    return np.linalg.norm(b - orc.spmv(A, x)) / np.linalg.norm(b)


# --------------------------------------------------------------------------- FCG
@pytest.mark.parametrize("fmt", ["csr", "ell", "sellp", "coo"])
def test_fcg_laplace2d_matches_oracle(g, orc, gen_mod, ctx, fmt):
    N = 64
    A = gen_mod.laplace2d(N)
    xs = gen_mod.uniform(2, N * N)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.fcg(A, b, tol=1e-10)
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = dev(np.zeros(N * N))
    info = g.fcg(M, dev(b), x, tol=1e-10, maxit=5000)
    assert info["status"] == g.OK, info
    assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    xg = host(x)
    assert relres(orc, A, b, xg) <= 1e-10
    kappa = (4 + 4 * math.cos(math.pi / (N + 1))) / (4 - 4 * math.cos(math.pi / (N + 1)))
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 2 * kappa * 1e-10


def test_fcg_block_jacobi_and_mixed(g, orc, gen_mod, ctx):
    N = 24
    A = gen_mod.laplace3d(N)
    n = N ** 3
    b = orc.spmv(A, gen_mod.uniform(5, n))
    rc, inv = orc.bj_invert(A, 8)
    rc, xo, info_o = orc.fcg(A, b, tol=1e-10, bj_inv=inv)
    M = g.Matrix.from_csr(*A)
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    x = dev(np.zeros(n))
    info = g.fcg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK and abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    assert relres(orc, A, b, host(x)) <= 1e-10
    # with a fixed SPD preconditioner FCG and CG agree up to rounding
    xc = dev(np.zeros(n))
    infoc = g.cg(M, dev(b), xc, tol=1e-10)
    assert abs(infoc["iterations"] - info["iterations"]) <= 1
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR, precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    x = dev(np.zeros(n))
    info = g.fcg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK and info["outer_iterations"] >= 2
    assert relres(orc, A, b, host(x)) <= 1e-10


def test_fcg_statuses(g, gen_mod, ctx):
    L = g.Matrix.from_csr(*gen_mod.laplace2d(32))
    info = g.fcg(L, dev(np.zeros(1024)), dev(np.ones(1024)))
    assert info["status"] == g.OK and info["iterations"] == 0
    info = g.fcg(L, dev(np.ones(1024)), dev(np.zeros(1024)), tol=1e-10, maxit=5)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 5
    D = g.Matrix.from_csr(np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32),
                          np.array([1.0, 2.0, -1.0, 3.0]))
    assert g.fcg(D, dev(np.ones(4)), dev(np.zeros(4)))["status"] == g.ERR_NOT_SPD


# --------------------------------------------------------------------------- CGS
@pytest.mark.parametrize("fmt", ["csr", "csr_merge", "coo", "ell", "hybrid", "sellp"])
def test_cgs_convdiff_matches_oracle(g, orc, gen_mod, ctx, fmt):
    A = gen_mod.convdiff2d(40, 0.5)
    n = 1600
    xs = gen_mod.uniform(8, n)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.cgs(A, b, tol=1e-10, maxit=2000)
    assert rc == orc.OK
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = dev(np.zeros(n))
    info = g.cgs(M, dev(b), x, tol=1e-10, maxit=2000)
    assert info["status"] == g.OK, info
    # no closed form for CGS iteration counts: they must stay close
    assert abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 10), (info, info_o)
    xg = host(x)
    true = relres(orc, A, b, xg)
    assert true <= 1e-9 and abs(info["true_rel_residual"] - true) <= 1e-12
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-6


def test_cgs_identity_and_breakdown(g, gen_mod, ctx):
    b = gen_mod.uniform(3, 10)
    I = g.Matrix.from_csr(np.arange(11, dtype=np.int32), np.arange(10, dtype=np.int32),
                          np.full(10, 2.5))
    x = dev(np.zeros(10))
    info = g.cgs(I, dev(b), x)
    assert info["status"] == g.OK and info["iterations"] == 1
    assert np.allclose(host(x), b / 2.5, rtol=1e-15, atol=0)
    B = g.Matrix.from_csr(np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.ones(2))
    assert g.cgs(B, dev(np.array([1.0, 0.0])), dev(np.zeros(2)))["status"] == g.ERR_BREAKDOWN
    L = g.Matrix.from_csr(*gen_mod.convdiff2d(20, 0.5))
    info = g.cgs(L, dev(np.ones(400)), dev(np.zeros(400)), maxit=3)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 3
    assert g.cgs(L, dev(np.zeros(400)), dev(np.ones(400)))["status"] == g.OK


# --------------------------------------------------------------------------- GMRES
@pytest.mark.parametrize("fmt", ["csr", "coo", "hybrid", "sellp"])
def test_gmres_convdiff_matches_oracle(g, orc, gen_mod, ctx, fmt):
    A = gen_mod.convdiff2d(40, 0.5)
    n = 1600
    xs = gen_mod.uniform(8, n)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.gmres(A, b, tol=1e-10, maxit=20000, m=20)
    assert rc == orc.OK
    ctx.set_solver_opts(krylov_dim=20)
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = dev(np.zeros(n))
    info = g.gmres(M, dev(b), x, tol=1e-10, maxit=20000)
    assert info["status"] == g.OK, info
    # classical Gram-Schmidt (twice when needed) against the oracle's modified
    # Gram-Schmidt: the same Krylov spaces, different rounding
    assert abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 20), (info, info_o)
    assert abs(info["outer_iterations"] - info_o["cycles"]) <= 1
    xg = host(x)
    assert relres(orc, A, b, xg) <= 1e-10
    assert abs(info["true_rel_residual"] - relres(orc, A, b, xg)) <= 1e-13
    assert np.linalg.norm(xg - xo) / np.linalg.norm(xo) <= 1e-7


def test_gmres_minimal_residual_steps(g, orc, ctx):
    """k steps without restart: the residual is the least-squares minimum over
    the Krylov space (numpy on an orthonormal Krylov basis), and x matches
    the oracle's k-step iterate."""
    rng = np.random.default_rng(23)
    n = 30
    D = np.eye(n) * 2 + rng.uniform(-1, 1, (n, n)) * 0.25
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    A = (rp, np.tile(np.arange(n, dtype=np.int32), n), D.ravel())
    b = rng.uniform(-1, 1, n)
    ctx.set_solver_opts(krylov_dim=30)
    M = g.Matrix.from_csr(*A)
    for k in range(1, 7):
        x = dev(np.zeros(n))
        info = g.gmres(M, dev(b), x, tol=1e-15, maxit=k)
        assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == k
        xg = host(x)
        K = np.stack([np.linalg.matrix_power(D, j) @ b for j in range(k)], 1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(D @ Q, b, rcond=None)
        rmin = np.linalg.norm(b - D @ (Q @ y))
        assert abs(np.linalg.norm(b - D @ xg) - rmin) <= 1e-10 * np.linalg.norm(b), k
        rc, xo, _ = orc.gmres(A, b, tol=1e-15, maxit=k, m=30)
        assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo), k
        assert abs(info["rel_residual"] - rmin / np.linalg.norm(b)) <= 1e-10


@pytest.mark.parametrize("m", [1, 5, 30, 128])
def test_gmres_restart_lengths_laplace(g, orc, gen_mod, ctx, m):
    """n = 65,536 (64 workgroups of the multi-vector passes), restart lengths
    from GMRES(1) to the largest supported."""
    N = 256 if m >= 30 else 32
    A = gen_mod.laplace2d(N)
    n = N * N
    b = orc.spmv(A, gen_mod.uniform(2, n))
    tol = 1e-8
    rc, xo, info_o = orc.gmres(A, b, tol=tol, maxit=4000, m=m)
    ctx.set_solver_opts(krylov_dim=m)
    M = g.Matrix.from_csr(*A)
    x = dev(np.zeros(n))
    info = g.gmres(M, dev(b), x, tol=tol, maxit=4000)
    assert info["status"] == (g.OK if rc == orc.OK else g.ERR_NOT_CONVERGED), (info, info_o)
    assert abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 20), (info, info_o)
    if rc == orc.OK:
        assert relres(orc, A, b, host(x)) <= tol


@pytest.mark.parametrize("m,maxit", [(5, 20000), (30, 20000), (64, 20000), (8, 37)])
def test_gmres_one_workgroup_matches_multikernel(g, orc, gen_mod, ctx, m, maxit):
    """Small CSR systems (n <= 4096, m <= 64) run the whole GMRES in one
    workgroup launch; the multi-kernel path (single_workgroup = 0) takes the
    same steps: equal iteration and cycle counts up to rounding, both
    solutions within the oracle's tolerance (maxit = 37 stops inside a
    cycle)."""
    A = gen_mod.convdiff2d(60, 0.5)
    n = 3600
    b = orc.spmv(A, gen_mod.uniform(9, n))
    rc, xo, info_o = orc.gmres(A, b, tol=1e-10, maxit=maxit, m=m)
    out = {}
    for single in (1, 0):
        ctx.set_solver_opts(krylov_dim=m, single_workgroup=single)
        M = g.Matrix.from_csr(*A)
        x = dev(np.zeros(n))
        out[single] = (g.gmres(M, dev(b), x, tol=1e-10, maxit=maxit), host(x))
    (i1, x1), (i0, x0) = out[1], out[0]
    want = g.OK if rc == orc.OK else g.ERR_NOT_CONVERGED
    assert i1["status"] == i0["status"] == want, (i1, i0, info_o)
    assert abs(i1["iterations"] - i0["iterations"]) <= max(2, i0["iterations"] // 50), (i1, i0)
    assert abs(i1["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 20), (i1, info_o)
    assert abs(i1["outer_iterations"] - i0["outer_iterations"]) <= 1
    if want == g.OK:
        assert relres(orc, A, b, x1) <= 1e-10
        assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-8
    else:
        assert i1["iterations"] == i0["iterations"] == maxit
        assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-10
        assert abs(i1["rel_residual"] - i0["rel_residual"]) <= 1e-10


def test_gmres_statuses(g, gen_mod, ctx):
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    Dm = g.Matrix.from_csr(np.arange(51, dtype=np.int32), np.arange(50, dtype=np.int32), d)
    bb = gen_mod.uniform(31, 50)
    x = dev(np.zeros(50))
    info = g.gmres(Dm, dev(bb), x, tol=1e-12)
    assert info["status"] == g.OK and info["iterations"] <= 3
    assert np.allclose(host(x), bb / d, rtol=1e-11, atol=0)
    L = g.Matrix.from_csr(*gen_mod.convdiff2d(20, 0.5))
    info = g.gmres(L, dev(np.zeros(400)), dev(np.ones(400)))
    assert info["status"] == g.OK and info["iterations"] == 0
    info = g.gmres(L, dev(np.ones(400)), dev(np.zeros(400)), maxit=7)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 7
    bn = np.ones(400)
    bn[5] = np.nan
    assert g.gmres(L, dev(bn), dev(np.zeros(400)))["status"] == g.ERR_BREAKDOWN
    for bad in (0, 129):
        with pytest.raises(g.GkoError):
            ctx.set_solver_opts(krylov_dim=bad)


# --------------------------------------------------------------------------- pipelined CG
@pytest.mark.parametrize("fmt", ["csr", "ell", "sellp", "coo"])
def test_pipecg_laplace2d_matches_oracle(g, orc, gen_mod, ctx, fmt):
    N = 64
    A = gen_mod.laplace2d(N)
    xs = gen_mod.uniform(2, N * N)
    b = orc.spmv(A, xs)
    rc, xo, info_o = orc.pipecg(A, b, tol=1e-10)
    M = g.Matrix.from_csr(*A).convert(fmt)
    x = dev(np.zeros(N * N))
    info = g.pipecg(M, dev(b), x, tol=1e-10, maxit=5000)
    assert info["status"] == g.OK, info
    assert abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    xg = host(x)
    assert relres(orc, A, b, xg) <= 1e-10
    kappa = (4 + 4 * math.cos(math.pi / (N + 1))) / (4 - 4 * math.cos(math.pi / (N + 1)))
    assert np.linalg.norm(xg - xs) / np.linalg.norm(xs) <= kappa * 1e-10


def test_pipecg_iterates_are_cg_iterates(g, orc, ctx):
    """k steps of the GPU's pipelined CG against the oracle's CG (not its
    pipelined CG): equal in exact arithmetic, with and without block-Jacobi."""
    rng = np.random.default_rng(41)
    n = 40
    G = rng.standard_normal((n, n))
    D = G @ G.T / n + np.eye(n)
    D = (D + D.T) / 2
    A = (np.arange(0, n * n + 1, n, dtype=np.int32), np.tile(np.arange(n, dtype=np.int32), n),
         D.ravel())
    b = rng.uniform(-1, 1, n)
    rc, inv = orc.bj_invert(A, 8)
    M = g.Matrix.from_csr(*A)
    for bs in (0, 8):
        if bs:
            ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
        for k in (1, 2, 3, 5, 10):
            x = dev(np.zeros(n))
            info = g.pipecg(M, dev(b), x, tol=1e-300, maxit=k)
            assert info["iterations"] == k
            r1, xc, _ = orc.cg(A, b, tol=1e-300, maxit=k, **({"bj_inv": inv, "bs": 8} if bs else {}))
            assert np.linalg.norm(host(x) - xc) <= 1e-11 * np.linalg.norm(xc), (bs, k)


def test_pipecg_block_jacobi_mixed_and_statuses(g, orc, gen_mod, ctx):
    N = 24
    A = gen_mod.laplace3d(N)
    n = N ** 3
    b = orc.spmv(A, gen_mod.uniform(5, n))
    rc, inv = orc.bj_invert(A, 8)
    rc, xo, info_o = orc.pipecg(A, b, tol=1e-10, bj_inv=inv)
    M = g.Matrix.from_csr(*A)
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    x = dev(np.zeros(n))
    info = g.pipecg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK and abs(info["iterations"] - info_o["iters"]) <= 2, (info, info_o)
    assert relres(orc, A, b, host(x)) <= 1e-10
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR, precond=g.PRECOND_BLOCK_JACOBI, block_size=8)
    x = dev(np.zeros(n))
    info = g.pipecg(M, dev(b), x, tol=1e-10)
    assert info["status"] == g.OK and info["outer_iterations"] >= 2
    assert relres(orc, A, b, host(x)) <= 1e-10
    ctx.set_solver_opts()
    L = g.Matrix.from_csr(*gen_mod.laplace2d(32))
    info = g.pipecg(L, dev(np.zeros(1024)), dev(np.ones(1024)))
    assert info["status"] == g.OK and info["iterations"] == 0
    info = g.pipecg(L, dev(np.ones(1024)), dev(np.zeros(1024)), tol=1e-10, maxit=5)
    assert info["status"] == g.ERR_NOT_CONVERGED and info["iterations"] == 5
    D = g.Matrix.from_csr(np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32),
                          np.array([1.0, 2.0, -1.0, 3.0]))
    rc, xd, info_d = orc.pipecg((np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32),
                                 np.array([1.0, 2.0, -1.0, 3.0])), np.ones(4))
    info = g.pipecg(D, dev(np.ones(4)), dev(np.zeros(4)))
    assert info["status"] == g.ERR_NOT_SPD and info["iterations"] == info_d["iters"]


# --------------------------------------------------------------------------- shared edge cases
def test_nonzero_initial_guess_and_long_restart(g, orc, gen_mod, ctx):
    A = gen_mod.convdiff2d(30, 0.5)
    n = 900
    b = orc.spmv(A, gen_mod.uniform(8, n))
    x0 = gen_mod.uniform(12, n)
    M = g.Matrix.from_csr(*A)
    ctx.set_solver_opts(krylov_dim=25)
    rc, xo, info_o = orc.gmres(A, b, x0=x0, tol=1e-10, maxit=5000, m=25)
    x = dev(x0.copy())
    info = g.gmres(M, dev(b), x, tol=1e-10, maxit=5000)
    assert info["status"] == g.OK and abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 20)
    assert relres(orc, A, b, host(x)) <= 1e-10
    rc, xo, info_o = orc.cgs(A, b, x0=x0, tol=1e-10, maxit=2000)
    x = dev(x0.copy())
    info = g.cgs(M, dev(b), x, tol=1e-10, maxit=2000)
    assert info["status"] == g.OK and abs(info["iterations"] - info_o["iters"]) <= max(3, info_o["iters"] // 10)
    # restart length above n: the Krylov space becomes invariant (h_{j+1,j} = 0)
    rng = np.random.default_rng(5)
    D = rng.uniform(-1, 1, (40, 40)) + 4 * np.eye(40)
    Ad = (np.arange(0, 1601, 40, dtype=np.int32), np.tile(np.arange(40, dtype=np.int32), 40), D.ravel())
    ctx.set_solver_opts(krylov_dim=128)
    bd = rng.uniform(-1, 1, 40)
    x = dev(np.zeros(40))
    info = g.gmres(g.Matrix.from_csr(*Ad), dev(bd), x, tol=1e-12)
    assert info["status"] == g.OK and info["iterations"] <= 40 and info["outer_iterations"] <= 2
    assert np.linalg.norm(D @ host(x) - bd) <= 1e-11 * np.linalg.norm(bd)


@pytest.mark.parametrize("solver", ["fcg", "pipecg", "cgs", "gmres"])
def test_solver_argument_checks(g, gen_mod, ctx, solver):
    import torch
    fn = getattr(g, solver)
    A = gen_mod.laplace2d(8)
    F = g.Matrix.from_csr(*A, dtype=torch.float32)
    with pytest.raises(g.GkoError) as e:
        fn(F, dev(np.ones(64)), dev(np.zeros(64)), raise_on_failure=True)
    assert e.value.status == g.ERR_UNSUPPORTED          # solvers take FP64 matrices
    R = g.Matrix.from_csr(np.array([0, 1, 2], np.int32), np.array([0, 2], np.int32), np.ones(2),
                          n_cols=3)
    with pytest.raises(g.GkoError) as e:
        fn(R, dev(np.ones(2)), dev(np.zeros(3)), raise_on_failure=True)
    assert e.value.status == g.ERR_DIM_MISMATCH
    M = g.Matrix.from_csr(*A)
    for tol in (0.0, float("inf")):
        with pytest.raises(g.GkoError) as e:
            fn(M, dev(np.ones(64)), dev(np.zeros(64)), tol=tol, raise_on_failure=True)
        assert e.value.status == g.ERR_INVALID_ARG


# ----------------------------------------------------------------- HIP graphs
def _solve_pair(g, ctx, solver, M, b, n, **opts):
    """The same solve with the polling interval replayed from a HIP graph and
    launched kernel by kernel: x and the iteration count."""
    out = []
    for graphs in (1, 0):
        ctx.set_solver_opts(graphs=graphs, single_workgroup=0, **opts)
        x = dev(np.zeros(n))
        info = getattr(g, solver)(M, dev(b), x, tol=1e-10, maxit=5000)
        out.append((host(x), info))
    return out


@pytest.mark.parametrize("fmt", ["csr", "csr_merge", "coo", "ell", "hybrid", "sellp"])
@pytest.mark.parametrize("solver", ["cg", "fcg", "pipecg"])
def test_graph_replay_matches_eager_spd(g, orc, gen_mod, ctx, solver, fmt):
    """CG, flexible and pipelined CG: the graph holds the eager path's kernels
    with the same arguments, so every replay (one per polling interval, with
    the host's convergence poll between them) gives the same bits."""
    A = gen_mod.laplace2d(100)
    n = 10000
    b = orc.spmv(A, gen_mod.uniform(21, n))
    M = g.Matrix.from_csr(*A).convert(fmt)
    (xg, ig), (xe, ie) = _solve_pair(g, ctx, solver, M, b, n, check_every=7)
    assert ig["status"] == g.OK and ie["status"] == g.OK
    assert ig["iterations"] == ie["iterations"] and ig["iterations"] > 7 * 10
    assert np.array_equal(xg, xe)
    assert relres(orc, A, b, xg) <= 1e-10


@pytest.mark.parametrize("mixed", [False, True], ids=["fp64", "mixed"])
def test_graph_replay_matches_eager_pcg(g, orc, gen_mod, ctx, mixed):
    A = gen_mod.laplace3d(24)
    n = 24 ** 3
    b = orc.spmv(A, gen_mod.uniform(22, n))
    M = g.Matrix.from_csr(*A).convert("sellp")
    (xg, ig), (xe, ie) = _solve_pair(
        g, ctx, "cg", M, b, n, precond=g.PRECOND_BLOCK_JACOBI, block_size=8,
        precision=g.PREC_MIXED_IR if mixed else g.PREC_FP64)
    assert ig["status"] == g.OK and ie["status"] == g.OK
    assert ig["iterations"] == ie["iterations"]
    assert ig["outer_iterations"] == ie["outer_iterations"]
    assert np.array_equal(xg, xe)


@pytest.mark.parametrize("fmt", ["csr", "coo", "ell", "sellp"])
@pytest.mark.parametrize("solver", ["bicgstab", "cgs"])
def test_graph_replay_matches_eager_nonsymmetric(g, orc, gen_mod, ctx, solver, fmt):
    A = gen_mod.convdiff2d(100, 0.5)
    n = 10000
    b = orc.spmv(A, gen_mod.uniform(23, n))
    M = g.Matrix.from_csr(*A).convert(fmt)
    (xg, ig), (xe, ie) = _solve_pair(g, ctx, solver, M, b, n)
    assert ig["status"] == g.OK and ie["status"] == g.OK
    assert ig["iterations"] == ie["iterations"]
    assert np.array_equal(xg, xe)
    assert relres(orc, A, b, xg) <= 1e-9


def test_graphs_option_validated(g, ctx):
    with pytest.raises(g.GkoError) as e:
        ctx.set_solver_opts(graphs=2)
    assert e.value.status == g.ERR_INVALID_ARG
    assert ctx.solver_opts()["graphs"] == 1
