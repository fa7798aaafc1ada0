"""Pins for the oracle's SpMV (Sec. 6.1 defines the operation and its cost).

The oracle is checked against things other than itself: exact rational
arithmetic and a dense brute-force matvec on tiny inputs, and the closed-form
eigenpairs of the Laplacian-type stencils that the workloads use.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

U = 2.0 ** -53


def gamma(k):
    return k * U / (1 - k * U)


def dense_of(A, n_cols=None):
    rp, col, val = A
    n = len(rp) - 1
    D = np.zeros((n, n if n_cols is None else n_cols))
    for i in range(n):
        for k in range(rp[i], rp[i + 1]):
            D[i, col[k]] = val[k]
    return D


def random_sparse(rng, n, m, density):
    """Nonsymmetric tiny CSR built directly in Python (no generator, no oracle)."""
    rp, col, val = [0], [], []
    for i in range(n):
        cols = sorted(j for j in range(m) if rng.random() < density)
        col += cols
        val += [rng.uniform(-1, 1) for _ in cols]
        rp.append(len(col))
    return (np.array(rp, np.int32), np.array(col, np.int32), np.array(val))


@pytest.mark.parametrize("seed", range(6))
def test_spmv_equals_dense_bruteforce_bitwise(orc, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 65))
    m = int(rng.integers(1, 65))
    A = random_sparse(rng, n, m, density=float(rng.uniform(0.02, 0.5)))
    D = dense_of(A, m)
    x = rng.uniform(-1, 1, m)
    y0 = rng.uniform(-1, 1, n)
    for alpha, beta in [(1.0, 0.0), (-0.75, 1.0), (2.5, -0.3)]:
        yd = []
        for i in range(n):
            s = 0.0
            for j in range(m):               # ascending j, plain float arithmetic
                s = s + float(D[i, j]) * float(x[j])
            yd.append(alpha * s if beta == 0.0 else alpha * s + beta * float(y0[i]))
        # rectangular case: the oracle takes x of length m
        y = orc.spmv(A, x, alpha, beta, y0)
        assert np.array_equal(y, np.array(yd)), (n, m, alpha, beta)


def test_spmv_transposed_operand_is_detected(orc):
    # a nonsymmetric pattern: A x and A^T x differ, and the oracle gives A x
    A = (np.array([0, 2, 3, 3], np.int32), np.array([0, 2, 1], np.int32), np.array([1.0, 2.0, 3.0]))
    x = np.array([1.0, 10.0, 100.0])
    assert list(orc.spmv(A, x)) == [1.0 + 200.0, 30.0, 0.0]


@pytest.mark.parametrize("seed", range(4))
def test_spmv_within_gamma_of_exact_rational(orc, seed):
    rng = np.random.default_rng(100 + seed)
    n, m = 40, 50
    A = random_sparse(rng, n, m, 0.4)
    x = rng.uniform(-1, 1, m) * 10.0 ** rng.integers(-3, 4, m)
    y0 = rng.uniform(-1, 1, n)
    alpha, beta = 1.5, -0.5
    rp, col, val = A
    exact = []
    for i in range(n):
        s = Fraction(0)
        for k in range(rp[i], rp[i + 1]):
            s += Fraction(float(val[k])) * Fraction(float(x[col[k]]))
        exact.append(Fraction(alpha) * s + Fraction(beta) * Fraction(float(y0[i])))
    y = orc.spmv(A, x, alpha, beta, y0)
    y2 = orc.spmv_dot2(A, x, alpha, beta, y0)
    absy = orc.spmv_absbound(A, x, alpha, beta, y0)
    for i in range(n):
        L = rp[i + 1] - rp[i]
        err = abs(Fraction(float(y[i])) - exact[i])
        assert err <= Fraction(gamma(L + 2) * absy[i]) + Fraction(1, 10 ** 300)
        # Dot2: nearly exact (a few ulps of the result plus u^2-level terms)
        err2 = abs(Fraction(float(y2[i])) - exact[i])
        assert err2 <= Fraction(4 * U * abs(float(exact[i])) + 4 * U * U * L * absy[i]) + Fraction(1, 10 ** 300)


def test_spmv_beta_zero_does_not_read_y(orc):
    A = (np.array([0, 1, 2], np.int32), np.array([0, 1], np.int32), np.array([2.0, 3.0]))
    y = orc.spmv(A, np.array([1.0, 1.0]), 1.0, 0.0, np.array([np.nan, np.inf]))
    assert list(y) == [2.0, 3.0]


def test_spmv_empty_rows_and_alpha_zero(orc):
    A = (np.array([0, 0, 2, 2], np.int32), np.array([0, 2], np.int32), np.array([1.0, 1.0]))
    y = orc.spmv(A, np.array([1.0, 2.0, 3.0]), 2.0, 3.0, np.array([1.0, 1.0, 1.0]))
    assert list(y) == [3.0, 2.0 * 4.0 + 3.0, 3.0]
    y = orc.spmv(A, np.array([1.0, 2.0, 3.0]), 0.0, 2.0, np.array([1.0, -1.0, 5.0]))
    assert list(y) == [2.0, -2.0, 10.0]


def _sines(N, k):
    i = np.arange(1, N + 1)
    return np.sin(i * k * math.pi / (N + 1))


def _check_eigpair(orc, A, v, lam, lam_max):
    Av = orc.spmv(A, v)
    res = np.max(np.abs(Av - lam * v))
    assert res <= 1e-13 * lam_max * np.max(np.abs(v)), res


@pytest.mark.parametrize("k", [1, 7, 30])
def test_laplace1d_eigenpairs(orc, gen_mod, k):
    N = 31
    A = gen_mod.laplace1d(N)
    lam = 2 - 2 * math.cos(k * math.pi / (N + 1))
    _check_eigpair(orc, A, _sines(N, k), lam, 4.0)


@pytest.mark.parametrize("j,k", [(1, 1), (3, 17), (64, 2)])
def test_laplace2d_eigenpairs(orc, gen_mod, j, k):
    N = 64
    A = gen_mod.laplace2d(N)
    # node index ix + N*iy, eigenvector sin(ix j pi/(N+1)) sin(iy k pi/(N+1))
    v = np.outer(_sines(N, k), _sines(N, j)).reshape(-1)
    lam = 4 - 2 * math.cos(j * math.pi / (N + 1)) - 2 * math.cos(k * math.pi / (N + 1))
    _check_eigpair(orc, A, v, lam, 8.0)


@pytest.mark.parametrize("ks", [(1, 1, 1), (2, 5, 11), (12, 1, 7)])
def test_laplace3d_eigenpairs(orc, gen_mod, ks):
    N = 12
    A = gen_mod.laplace3d(N)
    a, b, c = ks
    v = np.einsum("i,j,k->ijk", _sines(N, c), _sines(N, b), _sines(N, a)).reshape(-1)
    lam = 6 - sum(2 * math.cos(t * math.pi / (N + 1)) for t in ks)
    _check_eigpair(orc, A, v, lam, 12.0)


@pytest.mark.parametrize("ks", [(1, 1, 1), (3, 9, 2), (10, 10, 10)])
def test_stencil27_eigenpairs(orc, gen_mod, ks):
    # 27 I - T (x) T (x) T with T = tridiag(1, 1, 1): eigenvalues 27 - prod(1 + 2 cos)
    N = 10
    A = gen_mod.stencil27(N)
    a, b, c = ks
    v = np.einsum("i,j,k->ijk", _sines(N, c), _sines(N, b), _sines(N, a)).reshape(-1)
    lam = 27 - np.prod([1 + 2 * math.cos(t * math.pi / (N + 1)) for t in ks])
    _check_eigpair(orc, A, v, lam, 54.0)


def test_ninepoint_eigenpairs(orc, gen_mod):
    N = 20
    A = gen_mod.grid(N, N, kind="box")
    j, k = 4, 13
    v = np.outer(_sines(N, k), _sines(N, j)).reshape(-1)
    lam = 9 - (1 + 2 * math.cos(j * math.pi / (N + 1))) * (1 + 2 * math.cos(k * math.pi / (N + 1)))
    _check_eigpair(orc, A, v, lam, 18.0)


def test_paper_byte_model_golden():
    """The paper's SpMV bound: 16 B/entry COO -> BW/8 flop/s, 12 B/entry CSR -> BW/6."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_bounds.json")) as f:
        g = json.load(f)
    bpe = g["bytes_per_entry"]
    assert bpe["coo_fp64"] == 8 + 4 + 4 and bpe["csr_fp64"] == 8 + 4
    for row in g["gpus"]:
        csr_bound = row["bw_gbs"] / bpe["csr_fp64"] * 2
        # the paper's stated CSR bound and peak fractions follow from its byte model
        if "csr_bound_gflops" in row:
            assert abs(csr_bound - row["csr_bound_gflops"]) / row["csr_bound_gflops"] < 0.05
        if "csr_peak_gflops" in row and "csr_peak_frac" in row:
            assert abs(row["csr_peak_gflops"] / csr_bound - row["csr_peak_frac"]) < 0.05
