"""GPU parity of the SpMV family and the format conversions against the oracle.

SpMV (Sec. 6.1): every format, FP64 and FP32, on edge cases (empty rows and
runs of them, nnz = 0, a single dense row, rows much longer than a tile or a
chunk, rectangular shapes) and on small instances of the workload shapes.
Conversions are integer bookkeeping and must match the oracle's arrays byte
for byte."""
import numpy as np
import pytest

from gpu_util import assert_spmv_close, dev, host, tiny_cases, workload_cases

pytestmark = pytest.mark.gpu

FORMATS = ["csr", "csr_merge", "coo", "ell", "hybrid", "sellp"]


@pytest.fixture(scope="module")
def g():
    import paper_2011_08879_amd as g
    return g


@pytest.fixture(scope="module")
def cases(gen_mod):
    c = tiny_cases()
    c.update(workload_cases(gen_mod))
    return c


def make(g, case, f32=False):
    n, m, rp, col, val = case
    import torch
    return g.Matrix.from_csr(rp, col, val.astype(np.float32) if f32 else val, n_cols=m,
                             dtype=torch.float32 if f32 else torch.float64)


def ell_infeasible(case, vb=8):
    """The library refuses ELL when padded storage exceeds 4x the CSR storage."""
    n, m, rp, col, val = case
    K = int(np.diff(rp).max(initial=0))
    ld = (n + 63) // 64 * 64
    return K * ld * (vb + 4) > 4 * (len(col) * (vb + 4) + (n + 1) * 4)


def sellp_infeasible(case, vb=8):
    """SELL-P is refused by the same rule: padded slots above 4x the CSR storage."""
    n, m, rp, col, val = case
    lens = np.diff(rp).astype(np.int64)
    ns = (n + 63) // 64
    padded = np.zeros(ns * 64, np.int64)
    padded[:n] = lens
    slots = int(padded.reshape(ns, 64).max(axis=1).sum()) * 64 if ns else 0
    return slots * (vb + 4) > 4 * (len(col) * (vb + 4) + (n + 1) * 4)


def infeasible(fmt, case, vb=8):
    return ((fmt == "ell" and ell_infeasible(case, vb)) or
            (fmt == "sellp" and sellp_infeasible(case, vb)))


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
@pytest.mark.parametrize("fmt", FORMATS)
def test_spmv_parity(g, orc, gen_mod, cases, fmt, f32):
    import torch
    for name, case in cases.items():
        n, m, rp, col, val = case
        A = make(g, case, f32)
        if infeasible(fmt, case, 4 if f32 else 8):
            with pytest.raises(g.GkoError) as e:
                A.convert(fmt)
            assert e.value.status == g.ERR_UNSUPPORTED
            assert A.describe().format == "csr"
            continue
        A.convert(fmt)
        assert A.describe().format == fmt
        x = gen_mod.uniform(7, m)
        y0 = gen_mod.uniform(8, n)
        if f32:
            vals, x, y0 = (val.astype(np.float32).astype(np.float64), x.astype(np.float32).astype(np.float64),
                           y0.astype(np.float32).astype(np.float64))
        else:
            vals = val
        Ah = (rp, col, vals)
        tdt = torch.float32 if f32 else torch.float64
        lens = np.diff(rp)
        for alpha, beta in [(1.0, 0.0), (1.5, -0.5), (-1.0, 1.0)]:
            xd = dev(x, tdt)
            yd = dev(y0, tdt)
            if beta == 0.0:
                yd.fill_(float("nan"))   # beta = 0: y must not be read
            g.spmv(A, alpha, xd, beta, yd)
            y = host(yd)
            ref = orc.spmv_dot2(Ah, x, alpha, beta, y0)
            absy = orc.spmv_absbound(Ah, x, alpha, beta, y0)
            assert_spmv_close(y, ref, absy, lens, f32, "%s/%s a=%g b=%g" % (name, fmt, alpha, beta))
        A.close()


@pytest.mark.parametrize("fmt", FORMATS)
def test_spmv_deterministic(g, gen_mod, cases, fmt):
    import torch
    case = cases["lognormal_20k"]
    if fmt in ("ell", "sellp"):
        case = cases["stencil27_14"]
    n, m = case[0], case[1]
    A = make(g, case).convert(fmt)
    x = dev(gen_mod.uniform(3, m))
    outs = []
    for _ in range(4):
        y = torch.empty(n, dtype=torch.float64, device="cuda")
        g.spmv(A, 1.0, x, 0.0, y)
        outs.append(host(y).view(np.int64))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


def test_spmv_rejects_overlap(g, cases):
    import torch
    A = make(g, cases["laplace2d_64"])
    v = torch.zeros(4096 + 10, dtype=torch.float64, device="cuda")
    with pytest.raises(g.GkoError) as e:
        g.spmv(A, 1.0, v[:4096], 0.0, v[10:])
    assert e.value.status == g.ERR_INVALID_ARG


def test_create_rejects_malformed(g):
    import torch
    rp = np.array([0, 2, 1, 3], np.int32)          # decreasing offsets
    with pytest.raises(g.GkoError):
        g.Matrix.from_csr(rp, np.array([0, 1, 2], np.int32), np.ones(3))
    rp = np.array([0, 2, 3], np.int32)
    with pytest.raises(g.GkoError):                  # unsorted columns in row 0
        g.Matrix.from_csr(rp, np.array([1, 0, 1], np.int32), np.ones(3))
    with pytest.raises(g.GkoError):                  # column out of range
        g.Matrix.from_csr(rp, np.array([0, 1, 7], np.int32), np.ones(3), n_cols=3)
    # int64 row offsets are accepted
    A = g.Matrix.from_csr(np.array([0, 1, 2], np.int64), np.array([0, 1], np.int32), np.ones(2))
    assert A.describe().nnz == 2


def bits(a):
    return np.ascontiguousarray(a).view(np.int64 if a.dtype == np.float64 else np.int32)


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
def test_conversions_bit_exact(g, orc, cases, f32):
    for name, case in cases.items():
        n, m, rp, col, val = case
        vals = val.astype(np.float32) if f32 else val
        A = make(g, case, f32)
        Ah = (rp, col, vals.astype(np.float64))
        # COO
        A.convert("coo")
        s = A.export_storage()
        r, c, v = orc.csr_to_coo(Ah)
        assert np.array_equal(host(s["coo_row"]), r), name
        assert np.array_equal(host(s["coo_col"]), c), name
        assert np.array_equal(bits(host(s["coo_val"])), bits(v.astype(vals.dtype))), name
        # HYB
        A.convert("hybrid")
        s = A.export_storage()
        K, ld, ec, ev, tr, tc, tv = orc.csr_to_hyb(Ah, value_bytes=4 if f32 else 8)
        assert (s["K"], s["ld"]) == (K, ld), name
        assert np.array_equal(host(s["ell_col"]), ec), name
        assert np.array_equal(bits(host(s["ell_val"])), bits(ev.astype(vals.dtype))), name
        assert np.array_equal(host(s["coo_row"]), tr), name
        assert np.array_equal(host(s["coo_col"]), tc), name
        assert np.array_equal(bits(host(s["coo_val"])), bits(tv.astype(vals.dtype))), name
        # ELL
        if not ell_infeasible(case, 4 if f32 else 8):
            A.convert("ell")
            s = A.export_storage()
            K, ld, ec, ev = orc.csr_to_ell(Ah)
            assert (s["K"], s["ld"]) == (K, ld), name
            assert np.array_equal(host(s["ell_col"]), ec), name
            assert np.array_equal(bits(host(s["ell_val"])), bits(ev.astype(vals.dtype))), name
        # SELL-P
        if not sellp_infeasible(case, 4 if f32 else 8):
            A.convert("sellp")
            d = A.describe()
            s = A.export_sellp()
            w, sets, sc, sv = orc.csr_to_sellp(Ah)
            assert (s["slice"], d.sellp_slices, d.sellp_slots) == (64, len(w), sets[-1]), name
            assert np.array_equal(host(s["sets"]), sets), name
            assert np.array_equal(host(s["widths"]), w), name
            assert np.array_equal(host(s["col"]), sc), name
            assert np.array_equal(bits(host(s["val"])), bits(sv.astype(vals.dtype))), name
            vb = 4 if f32 else 8
            wide = [int(x) for x in w if x > 512]       # slices summed by column chunks
            items = sum((x + 255) // 256 for x in wide)
            assert d.sellp_wide_slices == len(wide), name
            extra = (len(wide) * 4 + (len(wide) + 1) * 4 + items * (8 + 64 * 8)) if wide else 0
            assert d.stored_bytes == sets[-1] * (vb + 4) + (len(w) + 1) * 8 + len(w) * 4 + extra, name
            B = A.clone()
            assert B.describe() == d
            sb = B.export_sellp()
            assert np.array_equal(host(sb["col"]), sc), name
            B.close()
        # merge, and back to CSR from whatever is stored
        for fmt in ["csr_merge", "coo", "hybrid", "sellp", "csr"]:
            if fmt == "sellp" and sellp_infeasible(case, 4 if f32 else 8):
                continue
            A.convert(fmt)
            erp, ecol, evl = (host(t) for t in A.export_csr())
            assert np.array_equal(erp, rp) and np.array_equal(ecol, col), (name, fmt)
            assert np.array_equal(bits(evl), bits(vals)), (name, fmt)
        d = A.describe()
        assert d.format == "csr" and d.nnz == len(col) and d.stored_bytes == (n + 1) * 4 + len(col) * (8 if f32 else 12)
        B = A.clone()
        assert B.describe() == d
        A.close()
        B.close()


def test_auto_picks_a_format(g, cases):
    A = make(g, cases["stencil27_14"])
    A.convert("auto")
    assert A.describe().format in g.SELECTOR_FORMATS


def test_sellp_pads_per_slice(g, orc):
    """One long row makes ELL pad every row to it; SELL-P pads only its slice."""
    rng = np.random.default_rng(77)
    n = 3000
    lens = rng.integers(1, 9, n)
    lens[1234] = 100
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(n, size=l, replace=False)) for l in lens]).astype(np.int32)
    val = rng.uniform(-1, 1, len(col))
    case = (n, n, rp, col, val)
    assert ell_infeasible(case) and not sellp_infeasible(case)
    A = make(g, case)
    with pytest.raises(g.GkoError):
        A.convert("ell")
    A.convert("sellp")
    d = A.describe()
    w, sets, sc, sv = orc.csr_to_sellp((rp, col, val))
    assert d.sellp_slots == sets[-1] and d.sellp_slots < 3 * len(col)   # ELL: 22x
    # SELL-P to every other format and back is bit-exact
    for fmt in ["coo", "sellp", "hybrid", "sellp", "csr_merge", "sellp"]:
        A.convert(fmt)
    s = A.export_sellp()
    assert np.array_equal(host(s["col"]), sc) and np.array_equal(bits(host(s["val"])), bits(sv))
    with pytest.raises(g.GkoError) as e:     # not stored as SELL-P
        A.convert("csr")
        A.export_sellp()
    assert e.value.status == g.ERR_INVALID_ARG


def test_csr_kernel_choice_and_parity(g, orc, gen_mod):
    """The CSR kernel follows the row-length rule (the LDS-staged row-per-thread
    kernel, with 1, 4 or 8 lanes per row, for rows of a mean up to 96 and at
    most 256 entries; a quarter-mean subwarp for longer regular rows; a
    mean-width subwarp plus the workgroup-per-row kernel for irregular rows),
    and each of these paths meets the SpMV bound against the oracle."""
    rng = np.random.default_rng(21)
    lens = list(rng.integers(1, 4, 700))
    lens[350] = 300
    rp = np.zeros(701, np.int32)
    rp[1:] = np.cumsum(lens)
    col = np.concatenate([np.sort(rng.choice(700, size=l, replace=False)) for l in lens]).astype(np.int32)
    cases = {
        "laplace2d": (gen_mod.laplace2d(40), 0, False),
        "banded_mean64": (gen_mod.banded(12, 3000, 64, 48, 80), 0, False),
        "banded_mean120": (gen_mod.banded(13, 3000, 128, 100, 140), 16, False),
        "banded_mean40": (gen_mod.banded(19, 3000, 40, 32, 48), 0, False),
        "stencil27_19": (gen_mod.stencil27(19), 0, False),
        "lognormal": (gen_mod.random_lognormal(4, 20000, max_len=3000), 16, True),
        "one_long_row": ((rp, col, rng.uniform(-1, 1, len(col))), 4, True),
    }
    for name, (A, kernel, has_long) in cases.items():
        M = g.Matrix.from_csr(*A)
        d = M.describe()
        lens = np.diff(A[0])
        assert d.csr_kernel == kernel, (name, d)
        if kernel == 0:   # lanes per row from the mean row length
            mean = len(A[1]) / (len(A[0]) - 1)
            assert d.csr_row_lanes == (8 if mean >= 56 else 4 if mean >= 12 else 1), (name, d)
        assert d.max_row_len == lens.max(), (name, d)
        assert (d.csr_long_rows > 0) == has_long, (name, d)
        if has_long:
            assert d.csr_long_rows == int((lens > max(4 * kernel, 64)).sum()), (name, d)
        n = len(A[0]) - 1
        x = gen_mod.uniform(7, n)
        y = dev(np.full(n, np.nan))
        g.spmv(M, 1.0, dev(x), 0.0, y)
        ref = orc.spmv_dot2(A, x, 1.0, 0.0, np.zeros(n))
        absy = orc.spmv_absbound(A, x, 1.0, 0.0, np.zeros(n))
        assert_spmv_close(host(y), ref, absy, lens, False, name)
        M.close()


def arrow_matrix(n, arms, seed):
    """SPD: diagonal 4 + |row degree|, a tridiagonal band, and rows/columns
    0..len(arms)-1 coupled to `arms[k]` random far columns (a few long rows)."""
    rng = np.random.default_rng(seed)
    ent = {}
    for i in range(n):
        for j in (i - 1, i + 1):
            if 0 <= j < n:
                ent[(i, j)] = -1.0
    for k, a in enumerate(arms):
        for j in rng.choice(np.arange(len(arms), n), size=a, replace=False):
            v = rng.uniform(-0.5, 0.5)
            ent[(k, int(j))] = v
            ent[(int(j), k)] = v
    rows = [[] for _ in range(n)]
    for (i, j), v in ent.items():
        rows[i].append((j, v))
    rp, col, val = [0], [], []
    for i in range(n):
        r = sorted(rows[i])
        diag = 4.0 + sum(abs(v) for _, v in r)
        r = sorted(r + [(i, diag)])
        col += [j for j, _ in r]
        val += [v for _, v in r]
        rp.append(len(col))
    return np.array(rp, np.int32), np.array(col, np.int32), np.array(val)


@pytest.mark.parametrize("f32", [False, True], ids=["f64", "f32"])
def test_sellp_wide_slices(g, orc, gen_mod, f32):
    """Slices made wide by a few long rows are summed by column chunks: parity
    of the product, an unchanged layout, and CG through the unfused path."""
    import torch
    n = 20000
    rp, col, val = arrow_matrix(n, [3000, 700, 1500], 5)
    case = (n, n, rp, col, val)
    assert not sellp_infeasible(case, 4 if f32 else 8)
    A = make(g, case, f32).convert("sellp")
    d = A.describe()
    assert d.sellp_wide_slices == 1                  # rows 0-2 share the first slice
    vals = val.astype(np.float32).astype(np.float64) if f32 else val
    w, sets, sc, sv = orc.csr_to_sellp((rp, col, vals))
    s = A.export_sellp()
    assert np.array_equal(host(s["col"]), sc) and np.array_equal(host(s["sets"]), sets)
    x = gen_mod.uniform(7, n)
    y0 = gen_mod.uniform(8, n)
    if f32:
        x, y0 = x.astype(np.float32).astype(np.float64), y0.astype(np.float32).astype(np.float64)
    tdt = torch.float32 if f32 else torch.float64
    for alpha, beta in [(1.0, 0.0), (1.5, -0.5)]:
        yd = dev(y0, tdt)
        g.spmv(A, alpha, dev(x, tdt), beta, yd)
        ref = orc.spmv_dot2((rp, col, vals), x, alpha, beta, y0)
        absy = orc.spmv_absbound((rp, col, vals), x, alpha, beta, y0)
        assert_spmv_close(host(yd), ref, absy, np.diff(rp), f32, "arrow/sellp")
    if not f32:
        b = orc.spmv((rp, col, val), gen_mod.uniform(2, n))
        rc, xo, info_o = orc.cg((rp, col, val), b, tol=1e-10)
        xg = dev(np.zeros(n))
        info = g.cg(A, dev(b), xg, tol=1e-10)
        assert info["status"] == g.OK and abs(info["iterations"] - info_o["iters"]) <= 2
        assert np.linalg.norm(b - orc.spmv((rp, col, val), host(xg))) <= 1e-10 * np.linalg.norm(b)
