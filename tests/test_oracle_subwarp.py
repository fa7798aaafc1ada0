"""Pins for the subwarp primitive emulation (Sec. 4 cooperative groups; the
xor-butterfly subgroup reduction of Sec. 5), checked by brute force over
every subwarp size and lane of a 64-wide wavefront."""
import random

import pytest

from oracle import subwarp as sw


@pytest.mark.parametrize("size", [1, 2, 4, 8, 16, 32, 64])
def test_masks_partition_the_wave(size):
    seen = 0
    for tid in range(256):
        m = sw.mask(tid, size)
        assert sw.popcount(m) == size
        off = sw.lane_offset(tid, size)
        assert m == sum(1 << (off + r) for r in range(size))
        assert off + sw.rank(tid, size) == tid % 64
        seen |= m
    assert seen == sw.FULL


@pytest.mark.parametrize("size", [1, 2, 4, 8, 16, 32, 64])
def test_ballot_any_all_bruteforce(size):
    rnd = random.Random(size)
    for density in (0.0, 0.1, 0.5, 0.9, 1.0):
        preds = [rnd.random() < density for _ in range(64)]
        for tid in range(64):
            off = sw.lane_offset(tid, size)
            group = preds[off:off + size]
            assert sw.sub_ballot(preds, tid, size) == sum(int(p) << r for r, p in enumerate(group))
            assert sw.sub_any(preds, tid, size) == any(group)
            assert sw.sub_all(preds, tid, size) == all(group)


@pytest.mark.parametrize("size", [1, 2, 4, 8, 16, 32, 64])
def test_butterfly_leaves_group_sum_in_every_lane(size):
    vals = [random.Random(7 * size).randint(-1000, 1000) for _ in range(64)]
    vals = [v + i for i, v in enumerate(vals)]
    out = sw.butterfly_sum(vals, size)
    for lane in range(64):
        off = (lane // size) * size
        assert out[lane] == sum(vals[off:off + size])
