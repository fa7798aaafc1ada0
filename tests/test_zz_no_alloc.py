"""gko_cg_solve_noalloc (CG with every work buffer in the library's static
scratch array) against gko_cg_solve: the same kernels, so the same iterates
bit for bit, on consecutive calls whose second input is smaller than the first
(the scratch keeps the previous call's contents), on the multi-kernel and the
single-workgroup paths and on a fused-product format; plus its limits."""
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


def _pair(g, orc, M, A, b, tol=1e-10):
    """(info, x) of gko_cg_solve and of gko_cg_solve_noalloc on the same system."""
    n = len(b)
    x_ref = dev(np.zeros(n))
    info_ref = g.cg(M, dev(b), x_ref, tol=tol)
    x_na = dev(np.zeros(n))
    info_na = g.cg_noalloc(M, dev(b), x_na, tol=tol)
    assert info_ref["status"] == g.OK and info_na["status"] == g.OK, (info_ref, info_na)
    xr, xn = host(x_ref), host(x_na)
    assert info_na["iterations"] == info_ref["iterations"]
    assert np.array_equal(xr.view(np.int64), xn.view(np.int64))
    true = np.linalg.norm(b - orc.spmv(A, xn)) / np.linalg.norm(b)
    assert true <= tol
    assert info_na["true_rel_residual"] == info_ref["true_rel_residual"]
    return info_na


def test_noalloc_matches_cg_on_shrinking_inputs(g, orc, gen_mod, ctx):
    # 1) 200^2 rows (multi-kernel), 2) 100^2 rows (multi-kernel, smaller, the
    # scratch still holds call 1's vectors), 3) 64^2 rows on one workgroup,
    # 4) 70^2 rows stored as SELL-P (the fused product) after the larger calls
    for N, fmt, single in ((200, "csr", 1), (100, "csr", 1), (64, "csr", 1), (70, "sellp", 0)):
        ctx.set_solver_opts(single_workgroup=single)
        A = gen_mod.laplace2d(N)
        b = orc.spmv(A, gen_mod.uniform(2, N * N))
        M = g.Matrix.from_csr(*A).convert(fmt)
        info = _pair(g, orc, M, A, b)
        assert info["iterations"] > 0
        M.close()


def test_noalloc_repeat_and_trivial_rhs(g, orc, gen_mod, ctx):
    A = gen_mod.laplace2d(96)
    n = 96 * 96
    M = g.Matrix.from_csr(*A)
    b = orc.spmv(A, gen_mod.uniform(3, n))
    xs = []
    for _ in range(2):
        x = dev(np.zeros(n))
        assert g.cg_noalloc(M, dev(b), x, tol=1e-10)["status"] == g.OK
        xs.append(host(x).view(np.int64))
    assert np.array_equal(xs[0], xs[1])
    x = dev(np.ones(n))
    info = g.cg_noalloc(M, dev(np.zeros(n)), x)
    assert info["status"] == g.OK and info["iterations"] == 0 and not host(x).any()


def test_noalloc_limits(g, gen_mod, ctx):
    # one row over the limit: rejected before any launch, x untouched
    n = g.CG_NOALLOC_MAX_ROWS + 1
    D = g.Matrix.from_csr(np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                          np.full(n, 2.0))
    x = dev(np.full(n, 7.0))
    info = g.cg_noalloc(D, dev(np.ones(n)), x)
    assert info["status"] == g.ERR_INVALID_ARG
    assert "no-allocation limit" in info["error"]
    assert np.all(host(x) == 7.0)
    # at the limit it runs (a diagonal system: one iteration)
    m = g.CG_NOALLOC_MAX_ROWS
    D2 = g.Matrix.from_csr(np.arange(m + 1, dtype=np.int32), np.arange(m, dtype=np.int32),
                           np.full(m, 2.0))
    x2 = dev(np.zeros(m))
    info = g.cg_noalloc(D2, dev(np.ones(m)), x2, tol=1e-12)
    assert info["status"] == g.OK and info["iterations"] == 1
    assert np.all(host(x2) == 0.5)
    # a preconditioner or mixed precision needs allocation
    A = g.Matrix.from_csr(*gen_mod.laplace2d(16))
    ctx.set_solver_opts(precond=g.PRECOND_BLOCK_JACOBI, block_size=4)
    assert g.cg_noalloc(A, dev(np.ones(256)), dev(np.zeros(256)))["status"] == g.ERR_UNSUPPORTED
    ctx.set_solver_opts(precision=g.PREC_MIXED_IR)
    assert g.cg_noalloc(A, dev(np.ones(256)), dev(np.zeros(256)))["status"] == g.ERR_UNSUPPORTED
