"""GPU parity of the persistent batched CG against the per-system oracle.

Systems follow the batch recipe (3-/5-point SPD stencils, sizes U{32..1024},
diagonal shift U[0.1, 2]); right-hand sides b = A x* come from the oracle's
SpMV.  FP64 batches run CG; FP32 batches run FP32 CG inside FP64 refinement
(the oracle's per-system refinement on the same FP32 values)."""
import math

import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


def rhs(orc, B, vals=None):
    vals = B.val if vals is None else vals
    b = np.empty_like(B.xstar)
    for i in range(B.nsys):
        r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
        rp, c, _ = B.system(i)
        k0, k1 = int(B.nnz_off[i]), int(B.nnz_off[i + 1])
        b[r0:r1] = orc.spmv((rp, c, vals[k0:k1]), B.xstar[r0:r1])
    return b


def kappa(B, i):
    m, s = int(B.m[i]), float(B.shift[i])
    if B.pattern[i] == 3:
        c = 2 * math.cos(math.pi / (m + 1))
        return (2 + s + c) / (2 + s - c)
    return (8 + s) / s


def test_batch_fp64_matches_oracle(g, orc, gen_mod):
    import torch
    B = gen_mod.batch_systems(300, master_seed=6)
    b = rhs(orc, B)
    rc, xo, it_o, rr_o = orc.batch_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val, b, tol=1e-10)
    assert rc == orc.OK
    G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val)
    for block, mode in ((64, "all"), (128, "all"), (256, "direction"), (256, "waves"),
                        (512, "waves")):
        G.block = block
        G.lds_mode = mode
        x = dev(np.full(B.xstar.shape, np.nan))
        st, it, rr = G.solve(dev(b), x, tol=1e-10)
        assert st == g.OK
        xg, itg, rrg = host(x), host(it), host(rr)
        assert np.all(np.abs(itg - it_o) <= 2), (block, np.abs(itg - it_o).max())
        assert np.all(rrg <= 1e-10)
        for i in range(B.nsys):
            r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
            rp, c, v = B.system(i)
            true = np.linalg.norm(b[r0:r1] - orc.spmv((rp, c, v), xg[r0:r1])) / np.linalg.norm(b[r0:r1])
            assert true <= 1e-10 and abs(true - rrg[i]) <= 1e-12
            err = np.linalg.norm(xg[r0:r1] - B.xstar[r0:r1]) / np.linalg.norm(B.xstar[r0:r1])
            assert err <= kappa(B, i) * 1e-10


def test_batch_fp32_refined_matches_oracle(g, orc, gen_mod):
    import torch
    B = gen_mod.batch_systems(200, master_seed=6)
    v32 = B.val.astype(np.float32)
    vals = v32.astype(np.float64)          # the FP32-stored matrix, exactly
    b = rhs(orc, B, vals)
    rc, xo, it_o, rr_o = orc.batch_ir_cg(B.row_off, B.nnz_off, B.row_ptr, B.col, vals, b, tol=1e-10)
    assert rc == orc.OK and np.all(rr_o <= 1e-10)
    G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, v32, dtype=torch.float32)
    for block, mode in ((G.block, G.lds_mode), (256, "waves"), (128, "waves")):
        G.block = block
        G.lds_mode = mode
        assert G.lds_mode == mode
        x = dev(np.zeros(B.xstar.shape))
        st, it, rr = G.solve(dev(b), x, tol=1e-10)
        assert st == g.OK
        xg, itg, rrg = host(x), host(it), host(rr)
        assert np.all(rrg <= 1e-10)
        # same refinement schedule; FP32 rounding may move each inner stop by a few steps
        assert np.all(np.abs(itg - it_o) <= np.maximum(6, it_o // 10)), np.abs(itg - it_o).max()
        for i in range(0, B.nsys, 7):
            r0, r1 = int(B.row_off[i]), int(B.row_off[i + 1])
            rp, c, _ = B.system(i)
            k0, k1 = int(B.nnz_off[i]), int(B.nnz_off[i + 1])
            true = np.linalg.norm(b[r0:r1] - orc.spmv((rp, c, vals[k0:k1]), xg[r0:r1])) / np.linalg.norm(b[r0:r1])
            assert true <= 1e-10


def test_batch_deterministic_and_autotune(g, orc, gen_mod):
    B = gen_mod.batch_systems(500, master_seed=11)
    b = rhs(orc, B)
    G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val)
    xs = []
    for _ in range(2):
        x = dev(np.zeros(B.xstar.shape))
        G.solve(dev(b), x)
        xs.append(host(x).view(np.int64))
    assert np.array_equal(xs[0], xs[1])
    x = dev(np.zeros(B.xstar.shape))
    blk, times = G.autotune(dev(b), x)
    assert blk in (64, 128, 256, 512) and G.block == blk
    assert all(t > 0 for t in times.values())
    assert times[(blk, G.lds_mode)] == min(times.values())
    # direction-only LDS fits FP64 systems of up to 4 * 256 rows at 256 threads, not at 64
    assert np.isfinite(times[(256, "direction")]) and np.isinf(times[(64, "direction")])
    assert np.isfinite(times[(256, "waves")]) and np.isinf(times[(64, "waves")])
    # every mode gives the oracle's solutions
    for mode in ("all", "direction", "waves"):
        G.block = 256
        G.lds_mode = mode
        x = dev(np.zeros(B.xstar.shape))
        st, it, rr = G.solve(dev(b), x)
        assert st == g.OK and G.lds_mode == mode
        assert float(host(rr).max()) <= 1e-10
        assert np.abs(host(x) - B.xstar).max() <= 1e-6 * np.abs(B.xstar).max()
    G.block = 64
    assert G.lds_mode == "all"
    for mode in ("direction", "waves"):
        with pytest.raises(g.GkoError):
            G.lds_mode = mode


def test_batch_autotune_cache(g, orc, gen_mod, tmp_path, monkeypatch):
    """gko_batch_autotune stores its choice in the on-disk cache under the
    device architecture and the batch's shape; a later batch of the same
    shape starts from it, one of another shape does not; an empty
    GKO_AUTOTUNE_CACHE turns the cache off."""
    path = tmp_path / "autotune"
    monkeypatch.setenv("GKO_AUTOTUNE_CACHE", str(path))
    B = gen_mod.batch_systems(200, master_seed=13)
    b = dev(rhs(orc, B))
    G = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val)
    blk, _ = G.autotune(b, dev(np.zeros(B.xstar.shape)))
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("batch_cg gfx950")
    key, val = lines[0].split(" = ")
    mode = g.BATCH_LDS_MODES.index(G.lds_mode)
    assert val == "%d %d" % (blk, mode)
    assert " f64 nsys=200 rows=%d nnz=%d " % (B.row_off[-1], B.nnz_off[-1]) in key
    # a stored choice other than the default is what a new batch of this shape takes
    other = 512 if blk != 512 else 256
    path.write_text("%s = %d 0\n" % (key, other))
    H = g.Batch(B.row_off, B.nnz_off, B.row_ptr, B.col, B.val)
    assert H.block == other and H.lds_mode == "all"
    # retuning replaces the line; a batch of another shape keeps its default
    G.autotune(b, dev(np.zeros(B.xstar.shape)))
    mode = g.BATCH_LDS_MODES.index(G.lds_mode)
    assert path.read_text().splitlines() == ["%s = %d %d" % (key, G.block, mode)]
    C = gen_mod.batch_systems(150, master_seed=13)
    default = 64 if int(C.m.max()) <= 256 else 128
    assert g.Batch(C.row_off, C.nnz_off, C.row_ptr, C.col, C.val).block == default
    monkeypatch.setenv("GKO_AUTOTUNE_CACHE", "")
    path.unlink()
    G.autotune(b, dev(np.zeros(B.xstar.shape)))
    assert not path.exists()


def test_batch_edge_cases_and_statuses(g, orc):
    import torch
    # one 1x1 system, one 2x2 SPD system, one indefinite diagonal system
    row_off = np.array([0, 1, 3, 5], np.int64)
    nnz_off = np.array([0, 1, 5, 7], np.int64)
    rp = np.array([0, 1, 0, 2, 4, 0, 1, 2], np.int32)
    col = np.array([0, 0, 1, 0, 1, 0, 1], np.int32)
    val = np.array([4.0, 2.0, -1.0, -1.0, 2.0, 1.0, -1.0])
    G = g.Batch(row_off, nnz_off, rp, col, val)
    b = np.array([8.0, 1.0, 1.0, 1.0, 1.0])
    x = dev(np.zeros(5))
    st, it, rr = G.solve(dev(b), x)
    assert st == g.ERR_NOT_SPD
    xg = host(x)
    assert xg[0] == 2.0 and np.allclose(xg[1:3], [1.0, 1.0], rtol=1e-12)
    # iteration cap: a 1024-row 3-point system cannot converge in 3 steps
    m = 1024
    rp = np.concatenate([[0], np.cumsum([2] + [3] * (m - 2) + [2])]).astype(np.int32)
    col = np.concatenate([[0, 1]] + [[i - 1, i, i + 1] for i in range(1, m - 1)] + [[m - 2, m - 1]]).astype(np.int32)
    val = np.concatenate([[2.1, -1.0]] + [[-1.0, 2.1, -1.0]] * (m - 2) + [[-1.0, 2.1]])
    G = g.Batch(np.array([0, m], np.int64), np.array([0, len(col)], np.int64), rp, col, val)
    x = dev(np.zeros(m))
    st, it, rr = G.solve(dev(np.ones(m)), x, tol=1e-10, maxit=3)
    assert st == g.ERR_NOT_CONVERGED and int(host(it)[0]) == 3 and float(host(rr)[0]) > 1e-10
    # malformed input and size limit
    with pytest.raises(g.GkoError):
        g.Batch(np.array([0, 2], np.int64), np.array([0, 2], np.int64), np.array([0, 1, 2], np.int32),
                np.array([0, 5], np.int32), np.ones(2))
    n_big = 3000
    with pytest.raises(g.GkoError):
        g.Batch(np.array([0, n_big], np.int64), np.array([0, n_big], np.int64),
                np.arange(n_big + 1, dtype=np.int32), np.arange(n_big, dtype=np.int32), np.ones(n_big))


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
def test_batch_wave_mode_statuses(g, orc, f32):
    """The wavefront mode on small and boundary systems: a 1x1, a 2x2 SPD, an
    indefinite diagonal system (NOT_SPD), a zero right-hand side (x = 0) and
    3-point systems of 255, 256 (a wavefront's limit) and 257 rows (the
    workgroup path), next to each other in one batch."""
    import torch
    sizes = [255, 256, 257]
    row_off, nnz_off, rps, cols, vals = [0], [0], [], [], []

    def add(rp, col, val):
        rps.append(np.asarray(rp, np.int32))
        cols.append(np.asarray(col, np.int32))
        vals.append(np.asarray(val, np.float64))
        row_off.append(row_off[-1] + len(rp) - 1)
        nnz_off.append(nnz_off[-1] + len(col))

    add([0, 1], [0], [4.0])
    add([0, 2, 4], [0, 1, 0, 1], [2.0, -1.0, -1.0, 2.0])
    for m in sizes + [64]:
        rp = np.concatenate([[0], np.cumsum([2] + [3] * (m - 2) + [2])])
        col = np.concatenate([[0, 1]] + [[i - 1, i, i + 1] for i in range(1, m - 1)] + [[m - 2, m - 1]])
        val = np.concatenate([[2.5, -1.0]] + [[-1.0, 2.5, -1.0]] * (m - 2) + [[-1.0, 2.5]])
        add(rp, col, val)
    add([0, 1, 2], [0, 1], [1.0, -1.0])
    nsys = len(rps)
    rp_all, col_all, val_all = np.concatenate(rps), np.concatenate(cols), np.concatenate(vals)
    rng = np.random.default_rng(3)
    b = rng.uniform(-1, 1, row_off[-1])
    zero = slice(row_off[5], row_off[6])          # the 64-row system gets b = 0
    b[zero] = 0.0
    b[row_off[6]:row_off[7]] = [0.1, 1.0]         # p.q = 0.01 - 1 < 0 at the first step
    if f32:
        val_all = val_all.astype(np.float32)
    G = g.Batch(np.array(row_off, np.int64), np.array(nnz_off, np.int64), rp_all, col_all, val_all,
                dtype=torch.float32 if f32 else torch.float64)
    G.block = 256
    G.lds_mode = "waves"
    assert G.lds_mode == "waves"
    x = dev(np.full(row_off[-1], np.nan))
    st, it, rr = G.solve(dev(b), x, tol=1e-10)
    assert st == g.ERR_NOT_SPD
    xg, rrg = host(x), host(rr)
    assert np.all(xg[zero] == 0.0) and rrg[5] == 0.0
    for i in range(nsys - 1):                     # every system but the indefinite one converged
        r0, r1 = row_off[i], row_off[i + 1]
        A = (rps[i], cols[i], val_all[nnz_off[i]:nnz_off[i + 1]].astype(np.float64))
        if i != 5:
            true = np.linalg.norm(b[r0:r1] - orc.spmv(A, xg[r0:r1])) / np.linalg.norm(b[r0:r1])
            assert true <= 1e-10 and rrg[i] <= 1e-10, (i, true, rrg[i])
