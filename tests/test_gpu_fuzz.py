"""Seeded random matrices across the kernels' tile boundaries: every format's
SpMV (FP64 and FP32) against the oracle's near-exact product, and the
conversion chain back to CSR bit for bit.  Sizes and row-length mixes are
drawn so that rows straddle COO's 1024-entry wave chunks, merge-path's
1024-item tiles, SELL-P's 64-row slices, the row-per-thread kernel's
2048-entry LDS chunks and 256- or 64-row tiles (one or four lanes per row)
and the long-row threshold of the subwarp kernel."""
import numpy as np
import pytest

from gpu_util import assert_spmv_close, dev, host

pytestmark = pytest.mark.gpu

FORMATS = ["csr", "csr_merge", "coo", "ell", "hybrid", "sellp"]


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


def random_case(seed):
    r = np.random.default_rng(1000 + seed)
    n = int(r.choice([1, 64, 65, 257, 1025, 4097, 20011, 70001, int(r.integers(2, 30000))]))
    m = int(r.choice([n, n, max(1, n // 3), 3 * n + 7]))
    kind = r.integers(0, 5)
    if kind == 0:      # short regular rows
        lens = r.integers(0, 9, n)
    elif kind == 1:    # lognormal with a heavy tail
        lens = np.minimum(np.round(np.exp(r.normal(2.0, 1.2, n))), m).astype(np.int64)
    elif kind == 2:    # mostly empty with a few long rows
        lens = np.where(r.random(n) < 0.05, r.integers(100, 5000, n), 0)
    elif kind == 3:    # uniform mid-length
        lens = r.integers(10, 70, n)
    else:              # runs of empty rows between dense-ish blocks
        lens = np.where((np.arange(n) // 97) % 3 == 0, 0, r.integers(1, 30, n))
    lens = np.minimum(lens, m).astype(np.int64)
    rp = np.zeros(n + 1, np.int64)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(r.choice(m, size=int(l), replace=False)) for l in lens]
                         + [np.zeros(0, np.int64)])
    val = r.uniform(-1, 1, int(rp[-1]))
    return n, m, rp.astype(np.int32), col.astype(np.int32), val


def feasible(fmt, n, rp, vb):
    lens = np.diff(rp).astype(np.int64)
    csr = int(rp[-1]) * (vb + 4) + (n + 1) * 4
    if fmt == "ell":
        return int(lens.max(initial=0)) * ((n + 63) // 64 * 64) * (vb + 4) <= 4 * csr
    if fmt == "sellp":
        ns = (n + 63) // 64
        padded = np.zeros(ns * 64, np.int64)
        padded[:n] = lens
        return int(padded.reshape(ns, 64).max(axis=1).sum()) * 64 * (vb + 4) <= 4 * csr
    return True


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
@pytest.mark.parametrize("seed", range(24))
def test_random_spmv_and_conversions(g, orc, gen_mod, seed, f32):
    import torch
    n, m, rp, col, val = random_case(seed)
    tdt = torch.float32 if f32 else torch.float64
    vals = val.astype(np.float32).astype(np.float64) if f32 else val
    x = gen_mod.uniform(30 + seed, m)
    y0 = gen_mod.uniform(60 + seed, n)
    if f32:
        x, y0 = x.astype(np.float32).astype(np.float64), y0.astype(np.float32).astype(np.float64)
    Ah = (rp, col, vals)
    lens = np.diff(rp)
    alpha, beta = 1.25, -0.75
    ref = orc.spmv_dot2(Ah, x, alpha, beta, y0)
    absy = orc.spmv_absbound(Ah, x, alpha, beta, y0)
    A = g.Matrix.from_csr(rp, col, val.astype(np.float32) if f32 else val, n_cols=m, dtype=tdt)
    try:
        for fmt in FORMATS:
            if not feasible(fmt, n, rp, 4 if f32 else 8):
                with pytest.raises(g.GkoError) as e:
                    A.convert(fmt)
                assert e.value.status == g.ERR_UNSUPPORTED
                continue
            A.convert(fmt)
            yd = dev(y0, tdt)
            g.spmv(A, alpha, dev(x, tdt), beta, yd)
            assert_spmv_close(host(yd), ref, absy, lens, f32, "seed %d n %d %s" % (seed, n, fmt))
            erp, ecol, evl = (host(t) for t in A.export_csr())
            assert np.array_equal(erp, rp) and np.array_equal(ecol, col), (seed, fmt)
            assert np.array_equal(evl.astype(np.float64), vals), (seed, fmt)
    finally:
        A.close()
