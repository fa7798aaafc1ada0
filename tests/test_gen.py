"""The seeded input generators: determinism, the published SplitMix64
definition, and the shapes of the workloads."""
import math

import numpy as np


def test_splitmix64_published_values(gen_mod):
    # SplitMix64 from state 0: the first output of the reference implementation
    # (state += 0x9E3779B97F4A7C15 then the two xor-shift-multiply mixes)
    assert gen_mod.splitmix64_first(0, 0) == 0xE220A8397B1DCDAF
    # stream (seed, k) starts from state seed*8 + k
    assert gen_mod.splitmix64_first(0, 1) != gen_mod.splitmix64_first(0, 0)


def test_uniform_deterministic_and_in_range(gen_mod):
    a, b = gen_mod.uniform(1, 1000), gen_mod.uniform(1, 1000)
    assert np.array_equal(a, b) and a.min() >= -1 and a.max() <= 1
    assert abs(a.mean()) < 0.1
    assert not np.array_equal(a, gen_mod.uniform(2, 1000))


def test_stencil_sizes(gen_mod):
    rp, col, val = gen_mod.laplace2d(64)
    assert len(rp) - 1 == 4096 and rp[-1] == 5 * 4096 - 4 * 64 == 20224
    rp, col, val = gen_mod.stencil27(16)
    assert rp[-1] == (3 * 16 - 2) ** 3
    assert set(np.diff(rp)) == {8, 12, 18, 27}
    rp, col, val = gen_mod.laplace3d(8)
    assert rp[-1] == 7 * 512 - 6 * 64
    for A in (gen_mod.laplace3d(5), gen_mod.stencil27(5), gen_mod.convdiff2d(9)):
        rp, col, val = A
        for i in range(len(rp) - 1):
            c = col[rp[i]:rp[i + 1]]
            assert np.all(np.diff(c) > 0)


def test_lognormal_workload_shape(gen_mod):
    lens = gen_mod.lognormal_lengths(4, 200000)
    assert lens.max() == 10000 and lens.min() >= 1
    assert 15.0 < lens.mean() < 17.5
    rp, col, val = gen_mod.random_rows(4, lens[:2000], 200000)
    for i in range(0, 2000, 97):
        c = col[rp[i]:rp[i + 1]]
        assert len(c) == lens[i] and np.all(np.diff(c) > 0) and c.min() >= 0 and c.max() < 200000


def test_batch_systems_shape(gen_mod):
    B = gen_mod.batch_systems(500)
    assert B.m.min() >= 32 and B.m.max() <= 1024
    assert set(B.pattern) == {3, 5}
    assert B.shift.min() >= 0.1 and B.shift.max() <= 2.0
    for i in range(0, 500, 37):
        rp, col, val = B.system(i)
        m = int(B.m[i])
        assert rp[0] == 0 and rp[-1] == len(col) and len(rp) == m + 1
        assert col.min() >= 0 and col.max() < m
        D = np.zeros((m, m))
        for r in range(m):
            D[r, col[rp[r]:rp[r + 1]]] = val[rp[r]:rp[r + 1]]
        assert np.array_equal(D, D.T)
        if B.pattern[i] == 5:
            w = math.ceil(math.sqrt(m))
            assert D[0, w] == -1.0 if w < m else True
