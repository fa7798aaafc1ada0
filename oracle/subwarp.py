"""ORACLE -- test infrastructure, not part of the product.

CPU emulation of the subwarp ("cooperative group") primitives of Sec. 4
(cooperative groups): contiguous subwarps of a given power-of-two Size inside a
wavefront, with

    Rank       = tid % Size
    LaneOffset = floor((tid % warpsize) / Size) * Size
    Mask       = (~0 >> (warpsize - Size)) << LaneOffset
    ballot(p)  = (wave_ballot(p) & Mask) >> LaneOffset
    any(p)     = (wave_ballot(p) & Mask) != 0
    all(p)     = (wave_ballot(p) & Mask) == Mask

and the xor-butterfly reduction of Sec. 5 (kernel programming): for bitmask =
1, 2, 4, ... < Size every lane adds the value of lane (lane ^ bitmask), which
leaves the subwarp sum in every lane.  Wavefronts are 64 wide here and lane
masks are 64-bit unsigned integers.
"""
from __future__ import annotations

WARPSIZE = 64
FULL = (1 << WARPSIZE) - 1


def rank(tid: int, size: int) -> int:
    return tid % size


def lane_offset(tid: int, size: int) -> int:
    return ((tid % WARPSIZE) // size) * size


def mask(tid: int, size: int) -> int:
    return ((FULL >> (WARPSIZE - size)) << lane_offset(tid, size)) & FULL


def wave_ballot(preds) -> int:
    """64-bit mask with bit l set when lane l's predicate holds."""
    assert len(preds) == WARPSIZE
    m = 0
    for lane, p in enumerate(preds):
        if p:
            m |= 1 << lane
    return m


def sub_ballot(preds, tid: int, size: int) -> int:
    return (wave_ballot(preds) & mask(tid, size)) >> lane_offset(tid, size)


def sub_any(preds, tid: int, size: int) -> bool:
    return (wave_ballot(preds) & mask(tid, size)) != 0


def sub_all(preds, tid: int, size: int) -> bool:
    return (wave_ballot(preds) & mask(tid, size)) == mask(tid, size)


def butterfly_sum(values, size: int):
    """Every lane ends with the sum over its subwarp, combined in butterfly order."""
    v = list(values)
    assert len(v) == WARPSIZE
    b = 1
    while b < size:
        v = [v[lane] + v[lane ^ b] for lane in range(WARPSIZE)]
        b <<= 1
    return v


def popcount(x: int) -> int:
    return bin(x & FULL).count("1")
