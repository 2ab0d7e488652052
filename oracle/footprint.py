"""Footprint assembly: a box as a set of aligned mipmap cubes.

ORACLE (test infrastructure only). Follows the appendix algorithm "Footprint
assembly in 3D" and Sec. "Fast Sub-Volume Queries" with Fig. "footprint":

1. Per axis (``footprint_1d``), the clipped range ``[i, i+di)`` is cut into
   aligned power-of-two steps: each step's level is the smaller of
   floor(log2(remaining extent)) and the number of trailing zero bits of the
   current start, and the start advances by 2^level.
   Readings of garbled or silent points: the printed "leading zero count" of
   the extent stands for floor(log2 extent) (the only reading that gives the
   figure's steps); the trailing-zero count of a start of 0 is unbounded; an
   origin at or past the volume gives no steps.
2. The tensor product of the per-axis step lists gives rectangular boxes; each
   is tessellated by cubes whose level is the smallest of its axes' levels,
   2^(level_axis - level) cubes along each axis (``assembly``). The cube's
   address at its level is (start_axis >> level) + offset; the start of each
   axis is the start of that axis's step (the printed pseudo-code never
   advances its running position; advancing it per step is the reading that
   reproduces the figure).
3. Each cube stands for 8^level voxels (2^level per axis in d dimensions).

``maximal_cubes`` is an independent brute-force definition of the same set:
every aligned cube inside the box whose parent cube is not inside the box.
"""
from __future__ import annotations

from collections import Counter

import numpy as np

_UNBOUNDED = 1 << 62


def _floor_log2(v: int) -> int:
    return int(v).bit_length() - 1


def _trailing_zeros(v: int) -> int:
    if v == 0:
        return _UNBOUNDED
    return (int(v) & -int(v)).bit_length() - 1


def footprint_1d(i: int, di: int, dim: int):
    """List of (start, level) steps covering [i, min(i+di, dim))."""
    i, di = int(i), int(di)
    di = min(i + di, int(dim)) - i
    steps = []
    while di > 0:
        a = _floor_log2(di)
        b = _trailing_zeros(i)
        lev = min(a, b)
        steps.append((i, lev))
        di -= 1 << lev
        i += 1 << lev
    return steps


def rectangles(p, dp, dims):
    """Tensor product of the per-axis step lists: list of (starts, levels) per rectangle."""
    lists = [footprint_1d(p[a], dp[a], dims[a]) for a in range(len(p))]
    out = [((), ())]
    for lst in lists:
        out = [(s + (st,), l + (lv,)) for (s, l) in out for (st, lv) in lst]
    return out


def assembly(p, dp, dims):
    """All cubes of the footprint as a list of (level, coords-at-level) in any dimension count."""
    cubes = []
    for starts, levels in rectangles(p, dp, dims):
        lev = min(levels)
        counts = [1 << (la - lev) for la in levels]
        base = [s >> lev for s in starts]
        for off in np.ndindex(*counts):
            cubes.append((lev, tuple(b + o for b, o in zip(base, off))))
    return cubes


def cube_count(p, dp, dims) -> int:
    """Number of cubes (samples) of the footprint, without enumerating them."""
    total = 0
    for _, levels in rectangles(p, dp, dims):
        lev = min(levels)
        total += 1 << sum(la - lev for la in levels)
    return total


def level_histogram(p, dp, dims) -> Counter:
    """Counter {level: number of cubes}."""
    return Counter(lev for lev, _ in assembly(p, dp, dims))


def maximal_cubes(p, dp, dims):
    """Brute force: aligned cubes inside the clipped box whose parent cube is not inside it."""
    d = len(p)
    lo = [int(p[a]) for a in range(d)]
    hi = [min(int(p[a]) + int(dp[a]), int(dims[a])) for a in range(d)]
    if any(h <= l for l, h in zip(lo, hi)):
        return []

    def inside(lev, c):
        return all(lo[a] <= (c[a] << lev) and ((c[a] + 1) << lev) <= hi[a] for a in range(d))

    out = []
    lev = 0
    while True:
        rng = [range(lo[a] >> lev, ((hi[a] - 1) >> lev) + 1) for a in range(d)]
        any_inside = False
        for c in np.ndindex(*[len(r) for r in rng]):
            cc = tuple(rng[a][c[a]] for a in range(d))
            if inside(lev, cc):
                any_inside = True
                parent = tuple(v >> 1 for v in cc)
                if not inside(lev + 1, parent):
                    out.append((lev, cc))
        if not any_inside:
            break
        lev += 1
    return out


def expected_cube_count(edge: int, samples: int, seed: int) -> float:
    """Mean cube count of an edge^3 box over seeded uniformly random origins far from the borders."""
    g = np.random.Generator(np.random.PCG64(seed))
    big = 1 << 30
    tot = 0
    for _ in range(samples):
        org = g.integers(0, 1 << 20, size=3) + (1 << 20)
        lists = [footprint_1d(int(o), edge, big) for o in org]
        lv = [np.array([s[1] for s in lst], dtype=np.int64) for lst in lists]
        lx, ly, lz = lv[0][:, None, None], lv[1][None, :, None], lv[2][None, None, :]
        m = np.minimum(np.minimum(lx, ly), lz)
        tot += int(np.sum(np.left_shift(1, lx + ly + lz - 3 * m)))
    return tot / samples
