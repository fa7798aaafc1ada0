"""Pins for the oracle's format conversions (CSR <-> COO / ELL / HYB / SELL-P).

Layouts are this library's definitions (the paper names the formats' role in
Sec. 6.1 but not their layout): COO row-major triplets; ELL column-major with
leading dimension n rounded up to 64 and padding col = -1, val = +0.0; HYB an
ELL part of width K* (the byte-minimising split) plus a row-major COO tail;
SELL-P slices of C rows, each padded to its own width and column-major
inside the slice (Anzt, Tomov and Dongarra 2014, unsorted, stride factor 1).
Pinned by a hand-worked example, brute force and round-trip identities.
"""
import numpy as np
import pytest


def bits(a):
    return np.ascontiguousarray(a, np.float64).view(np.int64)


# A 5 x 4 example worked by hand.
RP = np.array([0, 2, 2, 3, 6, 7], np.int32)
CI = np.array([0, 2, 1, 0, 1, 3, 3], np.int32)
VA = np.array([1.0, 2.0, 3.0, 4.0, 5.0, 6.0, 7.0])
A5 = (RP, CI, VA)


def test_hand_example_coo(orc):
    r, c, v = orc.csr_to_coo(A5)
    assert list(r) == [0, 0, 2, 3, 3, 3, 4]
    assert list(c) == list(CI) and list(v) == list(VA)


def test_hand_example_ell(orc):
    K, ld, ec, ev = orc.csr_to_ell(A5)
    assert (K, ld) == (3, 64)
    ec = ec.reshape(K, ld)
    ev = ev.reshape(K, ld)
    assert list(ec[0, :5]) == [0, -1, 1, 0, 3]
    assert list(ec[1, :5]) == [2, -1, -1, 1, -1]
    assert list(ec[2, :5]) == [-1, -1, -1, 3, -1]
    assert list(ev[0, :5]) == [1.0, 0.0, 3.0, 4.0, 7.0]
    assert list(ev[1, :5]) == [2.0, 0.0, 0.0, 5.0, 0.0]
    assert np.all(ec[:, 5:] == -1) and np.all(bits(ev[:, 5:]) == 0)   # +0.0 padding


def test_hand_example_hyb(orc):
    # cost(K) = 5*K*12 + 16*tail(K): K=0 -> 112, K=1 -> 108, K=2 -> 136, K=3 -> 180
    assert orc.hyb_width(A5, 8) == 1
    # FP32: cost(K) = 5*K*8 + 12*tail: 84, 76, 92, 120 -> K = 1
    assert orc.hyb_width(A5, 4) == 1
    K, ld, ec, ev, tr, tc, tv = orc.csr_to_hyb(A5)
    assert K == 1
    assert list(ec[:5]) == [0, -1, 1, 0, 3]
    assert list(tr) == [0, 3, 3] and list(tc) == [2, 1, 3] and list(tv) == [2.0, 5.0, 6.0]


def hyb_width_bruteforce(rp, value_bytes):
    lens = np.diff(rp).astype(np.int64)
    n = len(lens)
    best, best_cost = 0, None
    for K in range(int(lens.max(initial=0)) + 1):
        cost = n * K * (value_bytes + 4) + (value_bytes + 8) * int(np.maximum(lens - K, 0).sum())
        if best_cost is None or cost < best_cost:
            best, best_cost = K, cost
    return best


def matrices(gen_mod):
    yield "lognormal", gen_mod.random_lognormal(11, 3000, mean=6.0, sigma=1.2, max_len=400)
    yield "uniform0", gen_mod.uniform_random(12, 2000, 0, 9)          # has empty rows
    yield "banded", gen_mod.banded(13, 1500, 20, 1, 30)
    yield "stencil27", gen_mod.stencil27(9)
    yield "blockdiag", gen_mod.blockdiag(14, 700, 4, 40)
    yield "one_row", (np.array([0, 5], np.int32), np.arange(5, dtype=np.int32), np.ones(5))
    yield "all_empty", (np.zeros(4, np.int32), np.zeros(0, np.int32), np.zeros(0))


def test_hyb_width_matches_bruteforce(orc, gen_mod):
    for name, A in matrices(gen_mod):
        for vb in (8, 4):
            assert orc.hyb_width(A, vb) == hyb_width_bruteforce(A[0], vb), name


def test_hyb_width_special_cases(orc):
    # all rows of equal length L: ELL slots (12 B) beat COO entries (16 B) -> K* = L
    L, n = 7, 100
    rp = np.arange(n + 1, dtype=np.int32) * L
    A = (rp, np.tile(np.arange(L, dtype=np.int32), n), np.ones(n * L))
    assert orc.hyb_width(A, 8) == L
    # one dense row among empty ones: the whole row goes to the COO tail
    rp = np.zeros(n + 1, np.int32)
    rp[1:] = 50
    A = (rp, np.arange(50, dtype=np.int32), np.ones(50))
    assert orc.hyb_width(A, 8) == 0


def test_roundtrips_bit_exact(orc, gen_mod):
    for name, A in matrices(gen_mod):
        rp, ci, va = A
        n = len(rp) - 1
        r, c, v = orc.csr_to_coo(A)
        # the triplet multiset is the matrix
        assert np.array_equal(np.repeat(np.arange(n), np.diff(rp)), r), name
        back = orc.coo_to_csr(n, r, c, v)
        assert np.array_equal(back[0], rp) and np.array_equal(back[1], ci), name
        assert np.array_equal(bits(back[2]), bits(va)), name
        K, ld, ec, ev = orc.csr_to_ell(A)
        assert ld % 64 == 0 and ld >= n
        assert int((ec >= 0).sum()) == len(ci), name
        back = orc.hyb_to_csr(n, K, ld, ec, ev)
        assert np.array_equal(back[0], rp) and np.array_equal(back[1], ci), name
        assert np.array_equal(bits(back[2]), bits(va)), name
        K, ld, ec, ev, tr, tc, tv = orc.csr_to_hyb(A)
        assert int((ec >= 0).sum()) + len(tr) == len(ci), name
        back = orc.hyb_to_csr(n, K, ld, ec, ev, tr, tc, tv)
        assert np.array_equal(back[0], rp) and np.array_equal(back[1], ci), name
        assert np.array_equal(bits(back[2]), bits(va)), name


def test_formats_give_same_spmv(orc, gen_mod):
    """A product computed from each layout (plain numpy on the arrays) equals CSR's values."""
    A = gen_mod.random_lognormal(21, 800, mean=5.0, sigma=1.0, max_len=100)
    n = len(A[0]) - 1
    x = gen_mod.uniform(22, n)
    y = orc.spmv(A, x)
    K, ld, ec, ev, tr, tc, tv = orc.csr_to_hyb(A)
    yh = np.zeros(n)
    for j in range(K):
        c = ec[j * ld:j * ld + n]
        yh += np.where(c >= 0, ev[j * ld:j * ld + n] * x[np.maximum(c, 0)], 0.0)
    np.add.at(yh, tr, tv * x[tc])
    absy = orc.spmv_absbound(A, x)
    assert np.all(np.abs(yh - y) <= 1e-14 * absy.max())


# --------------------------------------------------------------------------- SELL-P
def test_hand_example_sellp(orc):
    # slices of C = 2 rows: {0,1} width 2, {2,3} width 3, {4, pad row} width 1
    w, sets, sc, sv = orc.csr_to_sellp(A5, 2)
    assert list(w) == [2, 3, 1]
    assert list(sets) == [0, 4, 10, 12]
    # slot (j, r) of slice s at sets[s] + j*C + r
    assert list(sc) == [0, -1, 2, -1,  1, 0, -1, 1, -1, 3,  3, -1]
    assert list(sv) == [1.0, 0.0, 2.0, 0.0,  3.0, 4.0, 0.0, 5.0, 0.0, 6.0,  7.0, 0.0]
    assert np.all(bits(sv[sc < 0]) == 0)                                # +0.0 padding


def sellp_layout_bruteforce(rp, C):
    lens = np.diff(rp).astype(np.int64)
    n = len(lens)
    ns = (n + C - 1) // C
    padded = np.zeros(ns * C, np.int64)
    padded[:n] = lens
    w = padded.reshape(ns, C).max(axis=1) if ns else np.zeros(0, np.int64)
    return w, np.concatenate([[0], np.cumsum(w * C)])


@pytest.mark.parametrize("C", [1, 2, 7, 64])
def test_sellp_layout_and_roundtrip(orc, gen_mod, C):
    for name, A in matrices(gen_mod):
        rp, ci, va = A
        n = len(rp) - 1
        w, sets, sc, sv = orc.csr_to_sellp(A, C)
        bw, bsets = sellp_layout_bruteforce(rp, C)
        assert np.array_equal(w, bw) and np.array_equal(sets, bsets), name
        assert len(sc) == sets[-1] and int((sc >= 0).sum()) == len(ci), name
        assert np.all(bits(sv[sc < 0]) == 0), name
        back = orc.sellp_to_csr(n, w, sets, sc, sv, C)
        assert np.array_equal(back[0], rp) and np.array_equal(back[1], ci), name
        assert np.array_equal(bits(back[2]), bits(va)), name


def test_sellp_special_cases(orc, gen_mod):
    A = gen_mod.random_lognormal(31, 500, mean=6.0, sigma=1.0, max_len=80)
    rp, ci, va = A
    # C = 1: every slice is one row without padding, so SELL-P is CSR itself
    w, sets, sc, sv = orc.csr_to_sellp(A, 1)
    assert np.array_equal(sets, rp.astype(np.int64))
    assert np.array_equal(sc, ci) and np.array_equal(bits(sv), bits(va))
    # n <= C: one slice, which is ELL with leading dimension C
    B = gen_mod.uniform_random(32, 50, 0, 9)
    w, sets, sc, sv = orc.csr_to_sellp(B, 64)
    K, ld, ec, ev = orc.csr_to_ell(B)
    assert (len(w), int(w[0]), ld) == (1, K, 64)
    assert np.array_equal(sc, ec) and np.array_equal(bits(sv), bits(ev))


def test_sellp_spmv_from_layout(orc, gen_mod):
    """y computed from the SELL-P arrays (plain numpy) equals CSR's product."""
    A = gen_mod.random_lognormal(33, 900, mean=5.0, sigma=1.0, max_len=120)
    n = len(A[0]) - 1
    x = gen_mod.uniform(34, n)
    C = 64
    w, sets, sc, sv = orc.csr_to_sellp(A, C)
    y = np.zeros(len(w) * C)
    for s in range(len(w)):
        blk_c = sc[sets[s]:sets[s + 1]].reshape(w[s], C)
        blk_v = sv[sets[s]:sets[s + 1]].reshape(w[s], C)
        y[s * C:(s + 1) * C] = np.where(blk_c >= 0, blk_v * x[np.maximum(blk_c, 0)], 0.0).sum(axis=0)
    ref = orc.spmv(A, x)
    assert np.all(np.abs(y[:n] - ref) <= 1e-14 * orc.spmv_absbound(A, x).max())
    assert np.all(y[n:] == 0.0)
