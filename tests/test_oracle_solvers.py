"""Pins for the oracle's Krylov solvers, block-Jacobi and mixed-precision IR.

The paper (Sec. 6.2) benchmarks memory-bound Krylov solvers built on SpMV but
does not write them out; the oracle follows the textbook algorithms (CG:
Hestenes-Stiefel / Saad Alg. 9.1; BiCGSTAB: van der Vorst 1992; flexible CG:
Notay 2000; CGS: Sonneveld 1989 / Saad Alg. 7.5; restarted GMRES: Saad and
Schultz 1986 / Saad Alg. 6.9; pipelined CG: Ghysels and Vanroose 2014).  Pinned by finite termination, closed-form
spectra (condition numbers, iteration bounds), manufactured solutions, exact
preconditioners, and each method's defining optimality or projection
property computed independently with dense linear algebra (GMRES: minimal
residual over the Krylov space; CGS: the squared BiCG residual polynomial;
FCG: the Galerkin solution over the preconditioned residuals; pipelined CG:
CG's iterates, step by step).
"""
import math

import numpy as np
import pytest


def diag_csr(d):
    n = len(d)
    return (np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.asarray(d, float))


def dense_to_csr(D):
    rp, col, val = [0], [], []
    for i in range(D.shape[0]):
        for j in range(D.shape[1]):
            if D[i, j] != 0:
                col.append(j)
                val.append(D[i, j])
        rp.append(len(col))
    return np.array(rp, np.int32), np.array(col, np.int32), np.array(val)


# --------------------------------------------------------------------------- BLAS-1
def test_dot_norm_closed_forms(orc):
    assert orc.dot(np.ones(1000), np.ones(1000)) == 1000.0
    assert orc.norm2(np.array([3.0, 4.0])) == 5.0
    x = np.arange(1, 101, dtype=float)
    assert orc.dot(x, x) == 100 * 101 * 201 / 6          # sum of squares, exact in FP64
    e = np.zeros(50)
    e[17] = 1.0
    y = np.linspace(-1, 1, 50)
    assert orc.dot(e, y) == y[17]
    assert orc.dot(np.zeros(0), np.zeros(0)) == 0.0


# --------------------------------------------------------------------------- CG
def test_cg_finite_termination_three_eigenvalues(orc, gen_mod):
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    b = gen_mod.uniform(31, 50)
    rc, x, info = orc.cg(diag_csr(d), b, tol=1e-12, maxit=100)
    assert rc == orc.OK
    assert info["iters"] <= 3 and info["true_relres"] <= 1e-12
    assert np.allclose(x, b / d, rtol=1e-12, atol=0)


@pytest.mark.parametrize("n", [1, 2, 5, 8])
def test_cg_tiny_spd_terminates_in_n(orc, n):
    rng = np.random.default_rng(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    D = Q @ np.diag(np.linspace(1.0, 4.0, n)) @ Q.T       # SPD, kappa = 4
    D = (D + D.T) / 2
    b = rng.uniform(-1, 1, n)
    rc, x, info = orc.cg(dense_to_csr(D), b, tol=1e-10, maxit=100)
    assert rc == orc.OK and info["iters"] <= n
    assert np.linalg.norm(D @ x - b) <= 1e-10 * np.linalg.norm(b) * 1.0001


def test_cg_config1_manufactured_and_iteration_bound(orc, gen_mod):
    N = 64
    A = gen_mod.laplace2d(N)
    xs = gen_mod.uniform(2, N * N)
    b = orc.spmv(A, xs)
    rc, x, info = orc.cg(A, b, tol=1e-10, maxit=5000)
    assert rc == orc.OK and info["true_relres"] <= 1e-10
    lmin = 4 - 4 * math.cos(math.pi / (N + 1))
    lmax = 4 + 4 * math.cos(math.pi / (N + 1))
    kappa = lmax / lmin
    assert abs(kappa - 1711.7) < 0.5
    bound = math.ceil(0.5 * math.sqrt(kappa) * math.log(2 / 1e-10))
    assert bound == 491 and info["iters"] <= bound
    err = np.linalg.norm(x - xs) / np.linalg.norm(xs)
    assert err <= kappa * info["true_relres"]


def test_cg_zero_rhs_nan_and_indefinite(orc, gen_mod):
    A = gen_mod.laplace1d(20)
    rc, x, info = orc.cg(A, np.zeros(20), x0=np.ones(20))
    assert rc == orc.OK and info["iters"] == 0 and np.all(x == 0)
    b = np.ones(20)
    b[3] = np.nan
    rc, x, info = orc.cg(A, b)
    assert rc == orc.BREAKDOWN
    rc, x, info = orc.cg(diag_csr([1.0, 2.0, -1.0, 3.0]), np.ones(4))
    assert rc == orc.NOT_SPD
    rc, x, info = orc.cg(gen_mod.laplace2d(32), np.ones(1024), tol=1e-10, maxit=5)
    assert rc == orc.NOT_CONVERGED and info["iters"] == 5


def test_cg_initial_guess_already_solution(orc, gen_mod):
    A = gen_mod.laplace1d(30)
    xs = gen_mod.uniform(5, 30)
    b = orc.spmv(A, xs)
    rc, x, info = orc.cg(A, b, x0=xs)
    assert rc == orc.OK and info["iters"] == 0


# --------------------------------------------------------------------------- block-Jacobi
def cheb_u(k, t):
    """Chebyshev polynomial of the second kind U_k(t)."""
    if k < 0:
        return 0.0
    a, b = 1.0, 2 * t
    if k == 0:
        return a
    for _ in range(k - 1):
        a, b = b, 2 * t * b - a
    return b


def tridiag_inverse(m, a):
    """Closed form inverse of tridiag(-1, a, -1) (order m): U_{i-1} U_{m-j} / U_m at a/2, i <= j."""
    t = a / 2
    inv = np.empty((m, m))
    for i in range(1, m + 1):
        for j in range(1, m + 1):
            lo, hi = min(i, j), max(i, j)
            inv[i - 1, j - 1] = cheb_u(lo - 1, t) * cheb_u(m - hi, t) / cheb_u(m, t)
    return inv


def test_bj_blocks_of_poisson_match_closed_form(orc, gen_mod):
    A = gen_mod.laplace3d(16)        # blocks of 8 rows along x: tridiag(-1, 6, -1)
    rc, inv = orc.bj_invert(A, 8)
    assert rc == orc.OK
    ref = tridiag_inverse(8, 6.0)
    assert np.max(np.abs(inv - ref[None])) <= 1e-15 * 8
    A = gen_mod.laplace2d(24)        # tridiag(-1, 4, -1)
    rc, inv = orc.bj_invert(A, 8)
    assert np.max(np.abs(inv - tridiag_inverse(8, 4.0)[None])) <= 1e-15 * 8


def test_bj_pivoting_short_last_block_and_identity(orc):
    rng = np.random.default_rng(7)
    n, bs = 21, 8                      # last block has 5 rows
    D = np.zeros((n, n))
    for b0 in range(0, n, bs):
        m = min(bs, n - b0)
        B = rng.uniform(-1, 1, (m, m))
        B[0, 0] = 0.0                  # forces a row exchange
        D[b0:b0 + m, b0:b0 + m] = B
    D[3, 15] = 0.5                     # off-block entries are ignored
    rc, inv = orc.bj_invert(dense_to_csr(D), bs)
    assert rc == orc.OK
    for k, b0 in enumerate(range(0, n, bs)):
        m = min(bs, n - b0)
        P = D[b0:b0 + m, b0:b0 + m] @ inv[k, :m, :m]
        assert np.max(np.abs(P - np.eye(m))) <= 1e-13 * np.linalg.cond(D[b0:b0 + m, b0:b0 + m])
    singular = dense_to_csr(np.diag([1.0, 0.0, 2.0]))
    assert orc.bj_invert(singular, 8)[0] == orc.BREAKDOWN


def test_pcg_exact_block_preconditioner_converges_in_one(orc):
    rng = np.random.default_rng(9)
    n, bs = 40, 8
    D = np.zeros((n, n))
    for b0 in range(0, n, bs):
        G = rng.standard_normal((bs, bs))
        D[b0:b0 + bs, b0:b0 + bs] = G @ G.T + bs * np.eye(bs)
    A = dense_to_csr(D)
    rc, inv = orc.bj_invert(A, bs)
    b = rng.uniform(-1, 1, n)
    rc, x, info = orc.cg(A, b, tol=1e-12, bj_inv=inv, bs=bs)
    assert rc == orc.OK and info["iters"] == 1


# --------------------------------------------------------------------------- BiCGSTAB
def test_bicgstab_convdiff_manufactured(orc, gen_mod):
    A = gen_mod.convdiff2d(40, 0.5)
    xs = gen_mod.uniform(8, 1600)
    b = orc.spmv(A, xs)
    rc, x, info = orc.bicgstab(A, b, tol=1e-10, maxit=2000)
    assert rc == orc.OK and info["true_relres"] <= 1e-10 * 1.01
    r = b - orc.spmv(A, x)
    assert np.linalg.norm(r) <= 1.01e-10 * np.linalg.norm(b)


def test_bicgstab_scaled_identity_one_step_and_spd(orc, gen_mod):
    b = gen_mod.uniform(3, 10)
    rc, x, info = orc.bicgstab(diag_csr([2.5] * 10), b)
    assert rc == orc.OK and info["iters"] == 1 and np.allclose(x, b / 2.5, rtol=1e-15, atol=0)
    A = gen_mod.laplace2d(64)
    xs = gen_mod.uniform(2, 4096)
    rc, x, info = orc.bicgstab(A, orc.spmv(A, xs), tol=1e-10)
    assert rc == orc.OK and info["true_relres"] <= 1.01e-10


def test_bicgstab_breakdown(orc):
    # A = [[0,1],[1,0]], b = e1: rhat.v = e1 . e2 = 0 at the first step
    A = (np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    rc, x, info = orc.bicgstab(A, np.array([1.0, 0.0]))
    assert rc == orc.BREAKDOWN


# --------------------------------------------------------------------------- mixed precision
def test_ir_cg_reaches_fp64_accuracy(orc, gen_mod):
    N = 16
    A = gen_mod.laplace3d(N)
    n = N ** 3
    xs = gen_mod.uniform(5, n)
    b = orc.spmv(A, xs)
    rc, inv = orc.bj_invert(A, 8)
    rc, x, info = orc.ir_cg(A, b, tol=1e-10, inner_tol=1e-5, bj_inv=inv)
    assert rc == orc.OK
    true = np.linalg.norm(b - orc.spmv(A, x)) / np.linalg.norm(b)
    assert true <= 1e-10
    lmin = 6 - 6 * math.cos(math.pi / (N + 1))
    lmax = 6 + 6 * math.cos(math.pi / (N + 1))
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= (lmax / lmin) * 1e-10
    # an FP32-only solve cannot get there: the refinement is what carries it
    assert 2 <= info["outer_iters"] <= 6
    rc64, x64, _ = orc.cg(A, b, tol=1e-10, bj_inv=inv)
    assert np.linalg.norm(x - x64) / np.linalg.norm(x64) <= 2 * (lmax / lmin) * 1e-10


def test_ir_cg_stagnation_reported(orc, gen_mod):
    A = gen_mod.laplace2d(32)
    b = orc.spmv(A, gen_mod.uniform(1, 1024))
    # one inner iteration per outer step cannot halve the residual every time
    rc, x, info = orc.ir_cg(A, b, tol=1e-10, max_outer=50, inner_tol=1e-5, max_inner=1)
    assert rc == orc.NOT_CONVERGED


def _scaled_blocks_spd(n, bs, seed):
    """An SPD matrix whose bs x bs diagonal blocks differ in scale by up to 1e4,
    each coupled weakly to the next block: block-Jacobi
    removes the scale spread, so with the preconditioner PCG needs a handful of
    steps and without it many more."""
    rng = np.random.default_rng(seed)
    D = np.zeros((n, n))
    for b0 in range(0, n, bs):
        m = min(bs, n - b0)
        G = rng.standard_normal((m, m))
        s = 10.0 ** rng.uniform(0, 4)
        D[b0:b0 + m, b0:b0 + m] = s * (G @ G.T / m + np.eye(m))
    for i in range(n - 1):
        if (i + 1) % bs == 0:            # couple neighbouring blocks, keep SPD
            c = 0.1 * math.sqrt(D[i, i] * D[i + 1, i + 1])
            D[i, i + 1] = D[i + 1, i] = -c
    return D


def _f32_data(A):
    """The FP32-rounded matrix: (row_ptr, col, float32 values) and the same
    values widened back to FP64, so the FP64 oracle runs on the data the FP32
    solve sees."""
    rp, col, val = A
    v32 = np.asarray(val, np.float64).astype(np.float32)
    return (rp, col, v32), (rp, col, v32.astype(np.float64))


def test_bj_apply_f32_is_the_rounded_blockwise_product(orc):
    """The FP32 preconditioner apply against numpy's dense block products of
    the same FP32 data in FP64: each entry within the FP32 rounding bound
    (bs + 1) u |D^-1| |r|; nonsymmetric blocks and a short last block, so a
    transposed block or a dropped entry fails."""
    rng = np.random.default_rng(11)
    bs, n = 8, 8 * 7 + 3
    nb = (n + bs - 1) // bs
    inv = np.zeros((nb, bs, bs), np.float32)
    for k in range(nb):
        m = min(bs, n - k * bs)
        inv[k, :m, :m] = rng.uniform(-1, 1, (m, m))
    r = rng.uniform(-1, 1, n).astype(np.float32)
    z = orc.bj_apply_f32(inv, r, bs)
    ref, bound = np.zeros(n), np.zeros(n)
    for k in range(nb):
        m = min(bs, n - k * bs)
        blk = inv[k, :m, :m].astype(np.float64)
        rb = r[k * bs:k * bs + m].astype(np.float64)
        ref[k * bs:k * bs + m] = blk @ rb
        bound[k * bs:k * bs + m] = np.abs(blk) @ np.abs(rb)
    u = 2.0 ** -24
    assert np.all(np.abs(z.astype(np.float64) - ref) <= (bs + 1) * u * bound)
    assert not np.allclose(inv[0], inv[0].T)


def test_pcg_f32_iterates_follow_fp64_pcg(orc):
    """The inner FP32 PCG takes the pinned FP64 PCG's steps: after k = 1..6
    iterations on the same FP32-rounded matrix, right-hand side and FP32
    block inverses, its iterate equals the FP64 one to FP32 accuracy.  A wrong
    beta fails from k = 2 on, a dropped or misapplied preconditioner from k = 1."""
    n, bs = 96, 8
    D = _scaled_blocks_spd(n, bs, 3)
    A32, A64 = _f32_data(dense_to_csr(D))
    rc, inv = orc.bj_invert(A64, bs)
    assert rc == orc.OK
    inv32 = inv.astype(np.float32)
    rhs = np.random.default_rng(4).uniform(-1, 1, n).astype(np.float32)
    for k in range(1, 7):
        st, d, it = orc.pcg_f32(A32, rhs, tol=1e-30, maxit=k, inv32=inv32, bs=bs)
        assert it == k and st == orc.NOT_CONVERGED
        rc, xk, info = orc.cg(A64, rhs.astype(np.float64), tol=1e-30, maxit=k,
                              bj_inv=inv32.astype(np.float64), bs=bs)
        assert info["iters"] == k
        err = np.linalg.norm(d - xk) / np.linalg.norm(xk)
        assert err <= 1e-4, (k, err)
    # without the preconditioner the first step already points elsewhere
    st, d1, _ = orc.pcg_f32(A32, rhs, tol=1e-30, maxit=1, inv32=None, bs=bs)
    rc, x1, _ = orc.cg(A64, rhs.astype(np.float64), tol=1e-30, maxit=1,
                       bj_inv=inv32.astype(np.float64), bs=bs)
    assert np.linalg.norm(d1 - x1) / np.linalg.norm(x1) > 1e-2


def test_pcg_f32_iteration_count_and_solution(orc):
    """To tau = 1e-5 the FP32 PCG stops within 2 iterations of the FP64 PCG on
    the same data, its solution meets the manufactured one within kappa times
    the requested reduction, and block-Jacobi is what makes it converge fast
    (without it the count is several times larger)."""
    n, bs = 200, 8
    D = _scaled_blocks_spd(n, bs, 5)
    A32, A64 = _f32_data(dense_to_csr(D))
    rc, inv = orc.bj_invert(A64, bs)
    inv32 = inv.astype(np.float32)
    xs = np.random.default_rng(6).uniform(-1, 1, n)
    rhs = orc.spmv(A64, xs).astype(np.float32)
    tau = 1e-5
    st, d, it = orc.pcg_f32(A32, rhs, tol=tau, maxit=1000, inv32=inv32, bs=bs)
    assert st == orc.OK
    rc, x64, info = orc.cg(A64, rhs.astype(np.float64), tol=tau, maxit=1000,
                           bj_inv=inv32.astype(np.float64), bs=bs)
    assert abs(it - info["iters"]) <= 2, (it, info)
    # the FP64 system that the FP32 data define, solved densely
    Ad = np.zeros((n, n))
    for i in range(n):
        Ad[i, A64[1][A64[0][i]:A64[0][i + 1]]] = A64[2][A64[0][i]:A64[0][i + 1]]
    xe = np.linalg.solve(Ad, rhs.astype(np.float64))
    kappa = np.linalg.cond(Ad)
    assert np.linalg.norm(d - xe) / np.linalg.norm(xe) <= kappa * 2 * tau
    st, d0, it0 = orc.pcg_f32(A32, rhs, tol=tau, maxit=5000, inv32=None, bs=bs)
    assert it0 >= 3 * it, (it0, it)


def test_ir_cg_first_inner_solve_is_fp64_pcg_to_inner_tol(orc, gen_mod):
    """The first refinement step solves A32 d = fp32(b / ||b||) from d = 0 to
    tau_0 = max(inner_tol, tol / 2): its inner count is the FP64 PCG's on that
    data within 2, for the block-scaled matrix and the 3D Laplacian."""
    cases = []
    D = _scaled_blocks_spd(160, 8, 7)
    cases.append(dense_to_csr(D))
    cases.append(gen_mod.laplace3d(12))
    for A in cases:
        n = A[0].shape[0] - 1
        xs = gen_mod.uniform(5, n)
        b = orc.spmv(A, xs)
        rc, inv = orc.bj_invert(A, 8)
        rc, x, info = orc.ir_cg(A, b, tol=1e-10, inner_tol=1e-5, bj_inv=inv)
        assert rc == orc.OK and len(info["inner_per_outer"]) == info["outer_iters"]
        assert sum(info["inner_per_outer"]) == info["inner_iters"]
        A32, A64 = _f32_data(A)
        rt = (b / np.linalg.norm(b)).astype(np.float32)
        rc, _, ref = orc.cg(A64, rt.astype(np.float64), tol=1e-5, maxit=1000,
                            bj_inv=inv.astype(np.float32).astype(np.float64), bs=8)
        assert abs(info["inner_per_outer"][0] - ref["iters"]) <= 2, (info, ref)


def test_ir_cg_total_budget(orc, gen_mod):
    """maxit caps the inner iterations summed over the outer steps."""
    A = gen_mod.laplace3d(12)
    b = orc.spmv(A, gen_mod.uniform(5, 12 ** 3))
    rc, inv = orc.bj_invert(A, 8)
    rc, x, full = orc.ir_cg(A, b, tol=1e-10, bj_inv=inv)
    assert rc == orc.OK
    cap = full["inner_iters"] - 3
    rc, x, info = orc.ir_cg(A, b, tol=1e-10, bj_inv=inv, maxit=cap)
    assert rc == orc.NOT_CONVERGED and info["inner_iters"] == cap
    assert info["inner_per_outer"][:-1] == full["inner_per_outer"][:len(info["inner_per_outer"]) - 1]


# --------------------------------------------------------------------------- batched
def test_batch_cg_closed_form_bounds(orc, gen_mod):
    B = gen_mod.batch_systems(40, master_seed=6)
    b = np.empty_like(B.xstar)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        b[r0:r1] = orc.spmv(B.system(i), B.xstar[r0:r1])
    rc, x, iters, rr = orc.batch_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val, b, tol=1e-10)
    assert rc == orc.OK and np.all(rr <= 1e-10)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        m, s = int(B.m[i]), float(B.shift[i])
        if B.pattern[i] == 3:
            kappa = (2 + s + 2 * math.cos(math.pi / (m + 1))) / (2 + s - 2 * math.cos(math.pi / (m + 1)))
            assert kappa <= 41
        else:
            kappa = (8 + s) / s            # Gershgorin bound, strictly diagonally dominant
        err = np.linalg.norm(x[r0:r1] - B.xstar[r0:r1]) / np.linalg.norm(B.xstar[r0:r1])
        assert err <= kappa * 1e-10
        # identical to a standalone solve of the same system
        rc1, x1, info = orc.cg(B.system(i), b[r0:r1], tol=1e-10)
        assert info["iters"] == iters[i] and np.array_equal(x1, x[r0:r1])


def test_batch_ir_cg_fp32_storage(orc, gen_mod):
    """Refinement around FP32 CG reaches 1e-10 on every system of an FP32-stored batch."""
    B = gen_mod.batch_systems(30, master_seed=6)
    vals = B.val.astype(np.float32).astype(np.float64)
    b = np.empty_like(B.xstar)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        rp, c, _ = B.system(i)
        k0, k1 = int(B.nnz_off[i]), int(B.nnz_off[i + 1])
        b[r0:r1] = orc.spmv((rp, c, vals[k0:k1]), B.xstar[r0:r1])
    rc, x, it, rr = orc.batch_ir_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, b, tol=1e-10)
    assert rc == orc.OK and np.all(rr <= 1e-10)
    rc64, x64, it64, rr64 = orc.batch_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, b, tol=1e-10)
    # the refined solution agrees with the FP64 solve of the same (FP32-valued) systems
    assert np.linalg.norm(x - x64) / np.linalg.norm(x64) <= 81 * 2e-10


# --------------------------------------------------------------------------- FCG
def test_fcg_equals_cg_with_fixed_spd_preconditioner(orc, gen_mod):
    """With a fixed SPD preconditioner z_{k+1}.r_k = 0, so FCG's beta is CG's
    (exact arithmetic): the same iterations and solution up to rounding."""
    A = gen_mod.laplace3d(12)
    n = 12 ** 3
    xs = gen_mod.uniform(5, n)
    b = orc.spmv(A, xs)
    rc, inv = orc.bj_invert(A, 8)
    for kw in ({}, {"bj_inv": inv, "bs": 8}):
        r1, x1, i1 = orc.cg(A, b, tol=1e-10, **kw)
        r2, x2, i2 = orc.fcg(A, b, tol=1e-10, **kw)
        assert r1 == r2 == orc.OK and abs(i1["iters"] - i2["iters"]) <= 1
        assert i2["true_relres"] <= 1e-10
        assert np.linalg.norm(x1 - x2) <= 1e-8 * np.linalg.norm(xs)


def test_fcg_finite_termination_and_exact_preconditioner(orc, gen_mod):
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    b = gen_mod.uniform(31, 50)
    rc, x, info = orc.fcg(diag_csr(d), b, tol=1e-12, maxit=100)
    assert rc == orc.OK and info["iters"] <= 3
    rng = np.random.default_rng(9)
    n, bs = 40, 8
    D = np.zeros((n, n))
    for b0 in range(0, n, bs):
        G = rng.standard_normal((bs, bs))
        D[b0:b0 + bs, b0:b0 + bs] = G @ G.T + bs * np.eye(bs)
    A = dense_to_csr(D)
    rc, inv = orc.bj_invert(A, bs)
    rc, x, info = orc.fcg(A, rng.uniform(-1, 1, n), tol=1e-12, bj_inv=inv, bs=bs)
    assert rc == orc.OK and info["iters"] == 1


def test_fcg_two_steps_are_the_galerkin_solution_for_a_nonsymmetric_preconditioner(orc):
    """FCG keeps consecutive directions A-conjugate for any preconditioner, so
    x_2 minimises the A-norm error over x_0 + span{z_0, z_1}.  CG's beta does
    not with a nonsymmetric preconditioner (checked too, so the pin tells the
    two coefficients apart)."""
    rng = np.random.default_rng(21)
    n, bs = 24, 8
    G = rng.standard_normal((n, n))
    D = G @ G.T / n + np.eye(n)                       # SPD, well conditioned
    A = dense_to_csr(D)
    blocks = []
    for b0 in range(0, n, bs):
        L = np.tril(D[b0:b0 + bs, b0:b0 + bs])        # lower triangle: nonsymmetric inverse
        blocks.append(np.linalg.inv(L))
    inv = np.concatenate([B.ravel() for B in blocks])

    def Minv(r):
        return np.concatenate([blocks[k] @ r[k * bs:(k + 1) * bs] for k in range(n // bs)])

    b = rng.uniform(-1, 1, n)
    z0 = Minv(b)
    x1 = z0 * (z0 @ b) / (z0 @ D @ z0)
    z1 = Minv(b - D @ x1)
    Z = np.stack([z0, z1], 1)
    x2 = Z @ np.linalg.solve(Z.T @ D @ Z, Z.T @ b)
    rc, xf, info = orc.fcg(A, b, tol=1e-15, maxit=2, bj_inv=inv, bs=bs)
    assert rc == orc.NOT_CONVERGED and info["iters"] == 2
    assert np.linalg.norm(xf - x2) <= 1e-12 * np.linalg.norm(x2)
    rc, xc, info = orc.cg(A, b, tol=1e-15, maxit=2, bj_inv=inv, bs=bs)
    assert np.linalg.norm(xc - x2) > 1e-6 * np.linalg.norm(x2)


# --------------------------------------------------------------------------- CGS
def bicg_poly_residual(D, r0, rh, k):
    """phi_k(A) r0 for BiCG's residual polynomial: phi_k(0) = 1 and
    phi_k(A) r0 orthogonal to span{rh, A^T rh, ..., (A^T)^{k-1} rh}."""
    K = [r0]
    for _ in range(k):
        K.append(D @ K[-1])                            # A^j r0, j = 0..k
    L = [rh]
    for _ in range(k - 1):
        L.append(D.T @ L[-1])
    # phi_k(A) r0 = r0 + sum_j c_j A^j r0;  L_i . (...) = 0
    M = np.array([[L[i] @ K[j] for j in range(1, k + 1)] for i in range(k)])
    c = np.linalg.solve(M, -np.array([L[i] @ r0 for i in range(k)]))
    coef = np.concatenate([[1.0], c])                  # phi_k(t) = sum coef_j t^j

    def apply(v):
        out, Ajv = np.zeros_like(v), v.copy()
        for j, cj in enumerate(coef):
            out += cj * Ajv
            Ajv = D @ Ajv
        return out
    return apply(apply(r0))                            # CGS: phi_k(A)^2 r0


def test_cgs_residual_is_the_squared_bicg_polynomial(orc):
    rng = np.random.default_rng(17)
    n = 20
    D = np.eye(n) * 3 + rng.uniform(-1, 1, (n, n)) * 0.3   # nonsymmetric, well conditioned
    A = dense_to_csr(D)
    b = rng.uniform(-1, 1, n)
    for k in (1, 2, 3):
        rc, x, info = orc.cgs(A, b, tol=1e-15, maxit=k)
        assert rc == orc.NOT_CONVERGED and info["iters"] == k
        r = b - D @ x
        ref = bicg_poly_residual(D, b, b, k)
        assert np.linalg.norm(r - ref) <= 1e-10 * np.linalg.norm(b), k


def test_cgs_finite_termination_identity_and_manufactured(orc, gen_mod):
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    b = gen_mod.uniform(31, 50)
    rc, x, info = orc.cgs(diag_csr(d), b, tol=1e-12, maxit=100)
    assert rc == orc.OK and info["iters"] <= 3
    b = gen_mod.uniform(3, 10)
    rc, x, info = orc.cgs(diag_csr([2.5] * 10), b)
    assert rc == orc.OK and info["iters"] == 1 and np.allclose(x, b / 2.5, rtol=1e-15, atol=0)
    A = gen_mod.convdiff2d(40, 0.5)
    xs = gen_mod.uniform(8, 1600)
    b = orc.spmv(A, xs)
    rc, x, info = orc.cgs(A, b, tol=1e-10, maxit=2000)
    assert rc == orc.OK and info["true_relres"] <= 1e-9   # recursive residual drifts in CGS
    # breakdown: A = [[0,1],[1,0]], b = e1 gives (A p).rhat = 0 at the first step
    A = (np.array([0, 1, 2], np.int32), np.array([1, 0], np.int32), np.array([1.0, 1.0]))
    rc, x, info = orc.cgs(A, np.array([1.0, 0.0]))
    assert rc == orc.BREAKDOWN


# --------------------------------------------------------------------------- GMRES
def test_gmres_minimises_the_residual_over_the_krylov_space(orc):
    """k GMRES steps (no restart) give min ||b - A x|| over x in K_k(A, b),
    computed here by least squares on an orthonormal Krylov basis."""
    rng = np.random.default_rng(23)
    n = 30
    D = np.eye(n) * 2 + rng.uniform(-1, 1, (n, n)) * 0.25
    A = dense_to_csr(D)
    b = rng.uniform(-1, 1, n)
    for k in range(1, 7):
        rc, x, info = orc.gmres(A, b, tol=1e-15, maxit=k, m=30)
        assert rc == orc.NOT_CONVERGED and info["iters"] == k and info["cycles"] == 1
        K = np.stack([np.linalg.matrix_power(D, j) @ b for j in range(k)], 1)
        Q, _ = np.linalg.qr(K)
        y, *_ = np.linalg.lstsq(D @ Q, b, rcond=None)
        xref = Q @ y
        rmin = np.linalg.norm(b - D @ xref)
        assert abs(np.linalg.norm(b - D @ x) - rmin) <= 1e-10 * np.linalg.norm(b), k
        assert np.linalg.norm(x - xref) <= 1e-8 * np.linalg.norm(xref), k
        # the Givens estimate is the residual of the least-squares solution
        assert abs(info["relres"] - rmin / np.linalg.norm(b)) <= 1e-10


def test_gmres_finite_termination_restarts_and_bad_m(orc, gen_mod):
    rng = np.random.default_rng(29)
    n = 10
    D = rng.uniform(-1, 1, (n, n)) + 3 * np.eye(n)
    rc, x, info = orc.gmres(dense_to_csr(D), rng.uniform(-1, 1, n), tol=1e-10, m=10)
    assert rc == orc.OK and info["iters"] <= n
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    b = gen_mod.uniform(31, 50)
    rc, x, info = orc.gmres(diag_csr(d), b, tol=1e-12, m=30)
    assert rc == orc.OK and info["iters"] <= 3
    A = gen_mod.convdiff2d(40, 0.5)
    xs = gen_mod.uniform(8, 1600)
    b = orc.spmv(A, xs)
    rc, x, info = orc.gmres(A, b, tol=1e-10, maxit=20000, m=20)
    assert rc == orc.OK and info["true_relres"] <= 1e-10 and info["cycles"] > 1
    rc, x, info = orc.gmres(A, b, tol=1e-10, maxit=50, m=20)
    assert rc == orc.NOT_CONVERGED and info["iters"] == 50
    rc, x, info = orc.gmres(A, b, m=0)
    assert rc == orc.BAD
    rc, x, info = orc.gmres(A, np.zeros(1600), m=5)
    assert rc == orc.OK and info["iters"] == 0 and not x.any()


# --------------------------------------------------------------------------- pipelined CG
def test_pipecg_iterates_are_cg_iterates(orc, gen_mod):
    """In exact arithmetic pipelined CG produces CG's iterates: after k steps
    (no stop) the two agree to rounding, with and without block-Jacobi."""
    rng = np.random.default_rng(41)
    n = 40
    G = rng.standard_normal((n, n))
    D = G @ G.T / n + np.eye(n)                        # SPD, kappa ~ 5
    A = dense_to_csr(D)
    b = rng.uniform(-1, 1, n)
    rc, inv = orc.bj_invert(A, 8)
    for kw in ({}, {"bj_inv": inv, "bs": 8}):
        for k in range(1, 11):
            r1, xc, i1 = orc.cg(A, b, tol=1e-300, maxit=k, **kw)
            r2, xp, i2 = orc.pipecg(A, b, tol=1e-300, maxit=k, **kw)
            assert i1["iters"] == i2["iters"] == k
            assert np.linalg.norm(xp - xc) <= 1e-12 * np.linalg.norm(xc), (k, kw.keys())


def test_pipecg_terminates_and_meets_manufactured_bounds(orc, gen_mod):
    d = np.array([1.0, 2.0, 3.0] * 17)[:50]
    b = gen_mod.uniform(31, 50)
    rc, x, info = orc.pipecg(diag_csr(d), b, tol=1e-12, maxit=100)
    assert rc == orc.OK and info["iters"] <= 3
    N = 64
    A = gen_mod.laplace2d(N)
    xs = gen_mod.uniform(2, N * N)
    b = orc.spmv(A, xs)
    rc, x, info = orc.pipecg(A, b, tol=1e-10)
    kappa = (4 + 4 * math.cos(math.pi / (N + 1))) / (4 - 4 * math.cos(math.pi / (N + 1)))
    assert rc == orc.OK and info["iters"] <= math.ceil(0.5 * math.sqrt(kappa) * math.log(2 / 1e-10))
    assert info["true_relres"] <= 1e-10
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= kappa * 1e-10
    D = (np.arange(5, dtype=np.int32), np.arange(4, dtype=np.int32), np.array([1.0, 2.0, -1.0, 3.0]))
    rc, x, info = orc.pipecg(D, np.ones(4))
    assert rc == orc.NOT_SPD
