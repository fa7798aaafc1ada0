"""Shared helpers of the GPU tests: host/device moves and the tolerance checks."""
import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def torch_mod():
    import torch
    return torch


def dev(a, dtype=None):
    torch = torch_mod()
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def host(t):
    torch_mod().cuda.synchronize()
    return t.detach().cpu().numpy()


def tiny_cases():
    """Edge-case CSR matrices built directly (n, m, row_ptr, col, val)."""
    rng = np.random.default_rng(1234)
    cases = {}

    def from_lens(lens, m, seed):
        r = np.random.default_rng(seed)
        rp = np.zeros(len(lens) + 1, np.int32)
        rp[1:] = np.cumsum(lens)
        col = np.concatenate([np.sort(r.choice(m, size=l, replace=False)) for l in lens]
                             ) if sum(lens) else np.zeros(0, np.int64)
        val = r.uniform(-1, 1, int(sum(lens)))
        return rp, col.astype(np.int32), val

    cases["one_entry"] = (1, 1) + (np.array([0, 1], np.int32), np.array([0], np.int32), np.array([2.5]))
    cases["one_empty_row"] = (1, 3) + (np.array([0, 0], np.int32), np.zeros(0, np.int32), np.zeros(0))
    cases["all_empty"] = (100, 100) + (np.zeros(101, np.int32), np.zeros(0, np.int32), np.zeros(0))
    lens = [0] * 70 + list(rng.integers(0, 5, 200)) + [0] * 500 + list(rng.integers(1, 4, 100)) + [0] * 65
    cases["empty_runs"] = (len(lens), 400) + from_lens(lens, 400, 1)
    lens = list(rng.integers(1, 3, 300))
    lens[150] = 300
    cases["one_dense_row"] = (300, 300) + from_lens(lens, 300, 2)
    lens = list(rng.integers(0, 6, 3000))
    lens[7] = 5000
    lens[1500] = 4100
    lens[2999] = 4500
    cases["long_rows"] = (3000, 6000) + from_lens(lens, 6000, 3)
    lens = list(rng.integers(0, 40, 2000))
    cases["rect_wide"] = (2000, 5000) + from_lens(lens, 5000, 4)
    lens = list(rng.integers(0, 3, 5000))
    cases["rect_tall"] = (5000, 40) + from_lens(lens, 40, 5)
    return cases


def workload_cases(gen):
    cases = {}
    rp, c, v = gen.laplace2d(64)
    cases["laplace2d_64"] = (len(rp) - 1, len(rp) - 1, rp, c, v)
    rp, c, v = gen.stencil27(14)
    cases["stencil27_14"] = (len(rp) - 1, len(rp) - 1, rp, c, v)
    rp, c, v = gen.random_lognormal(4, 20000, max_len=3000)
    cases["lognormal_20k"] = (len(rp) - 1, len(rp) - 1, rp, c, v)
    rp, c, v = gen.laplace3d(24)
    cases["laplace3d_24"] = (len(rp) - 1, len(rp) - 1, rp, c, v)
    return cases


def assert_spmv_close(y, y_ref, absy, lens, f32: bool, what=""):
    """Per-entry rounding bound of a length-L sum in any order plus the final
    alpha/beta combination: |y - y_ref| <= (L + 5) u absy (u = unit roundoff
    of the computing precision; y_ref is near exact: FP64 on the same inputs).
    FP64 additionally meets the normwise 1e-14 bound relative to max |A||x|."""
    u = U32 if f32 else U64
    d = np.abs(y.astype(np.float64) - y_ref)
    bound = (lens.astype(np.float64) + 5.0) * u * absy
    bad = np.nonzero(d > bound)[0]
    assert bad.size == 0, "%s: %d entries outside the rounding bound, first %s: %r vs %r" % (
        what, bad.size, bad[:5], y[bad[:5]], y_ref[bad[:5]])
    if not f32 and absy.size:
        assert d.max() <= 1e-14 * max(absy.max(), np.finfo(float).tiny), what
