"""Greedy factorization of mixtures into linear interpolations.

ORACLE (test infrastructure only). Follows Sec. "Compression" (the two greedy pair scores, Eqs.
greedy1 and greedy2) and Sec. "Implementation Details" (maximum search with the cutoff tau), in
plain Python on small inputs, recomputing the scores from scratch for every pick of stage 1.

Readings taken here:
- A mixture is a vector of integer voxel counts; factoring the pair (i, j) out of h replaces
  components i and j by one component, the node (h_i e_i + h_j e_j) / (h_i + h_j), with count
  h_i + h_j (Fig. "factorization": the first node mixes e_1 and e_2 in the ratio of m's entries).
  Two mixtures re-use one node when they factor the same pair in the same ratio (Fig. "DAG").
- Nodes are stored as (a, b, w) with node = (1 - w) a + w b, a the heavier part (ties: the lower
  ID) and w the exact fraction of b.
- phi1(i, j): number of mixtures holding both; phi2(i, j): over those mixtures, ||h||_0 - 1 if
  that exceeds 2, else 2. The pick is the pair of largest score; ties go to the smallest (i, j).
- Stage 1 runs the global maximum search over the mixtures with more than tau components,
  factoring the picked pair out of every such mixture holding both; a mixture leaves stage 1 as
  soon as it has tau components or fewer. Stage 2 takes the remaining mixtures in scanline order
  and factors each down to one component, each time by its own pair of largest score, the scores
  counted over all mixtures not yet down to one component.
- The mixtures are the distinct normalized histograms of the mip voxels of levels >= 1 that hold
  two segments or more, in scanline order of first appearance (level by level, x fastest).
"""
from __future__ import annotations

from math import gcd

import numpy as np

from . import mipmap


def phi(mixtures, strategy: str) -> dict:
    """{(i, j): score} over the given mixtures (dicts node -> count), i < j."""
    out = {}
    for h in mixtures:
        n = len(h)
        if n < 2:
            continue
        w = 1 if strategy == "occurrence" else (n - 1 if n > 2 else 2)
        keys = sorted(h)
        for x in range(n):
            for y in range(x + 1, n):
                out[(keys[x], keys[y])] = out.get((keys[x], keys[y]), 0) + w
    return out


def _best(scores: dict, allowed=None):
    best = None
    for k, s in scores.items():
        if allowed is not None and k not in allowed:
            continue
        if best is None or s > best[1] or (s == best[1] and k < best[0]):
            best = (k, s)
    return best


class _Dag:
    def __init__(self, nseg):
        self.nseg = nseg
        self.nodes = []          # (a, b, wn, wd) of node nseg + k
        self.index = {}

    def node(self, i, ci, j, cj):
        if ci > cj or (ci == cj and i < j):
            a, b, wn = i, j, cj
        else:
            a, b, wn = j, i, ci
        wd = ci + cj
        g = gcd(wn, wd)
        key = (a, b, wn // g, wd // g)
        if key not in self.index:
            self.index[key] = self.nseg + len(self.nodes)
            self.nodes.append(key)
        return self.index[key]

    def factor(self, h: dict, i, j):
        ci, cj = h.pop(i), h.pop(j)
        n = self.node(i, ci, j, cj)
        h[n] = ci + cj
        return n


def factorize(nseg: int, mixtures, strategy: str = "reduction", tau: int = 3):
    """Greedy factorization. mixtures: list of {source: count}. Returns (nodes, roots, picks):
    nodes [(a, b, wn, wd)] for IDs nseg, nseg + 1, ...; roots[m] = node of mixture m; picks = the
    pairs stage 1 chose, in order."""
    mix = [dict(h) for h in mixtures]
    dag = _Dag(nseg)
    stage1 = [len(h) >= 2 and len(h) > tau for h in mix]
    picks = []
    while True:
        active = [h for h, s in zip(mix, stage1) if s]
        best = _best(phi(active, strategy))
        if best is None or best[1] <= 0:
            break
        (i, j), _ = best
        picks.append((i, j))
        for m, h in enumerate(mix):
            if stage1[m] and i in h and j in h:
                dag.factor(h, i, j)
                if len(h) <= tau or len(h) < 2:
                    stage1[m] = False
    scores = phi([h for h in mix if len(h) >= 2], strategy)
    for h in mix:
        while len(h) >= 2:
            keys = sorted(h)
            own = {(keys[x], keys[y]) for x in range(len(keys)) for y in range(x + 1, len(keys))}
            (i, j), _ = _best({k: scores.get(k, 0) for k in own})
            for k, s in phi([h], strategy).items():
                scores[k] -= s
            dag.factor(h, i, j)
            for k, s in phi([h], strategy).items():
                scores[k] = scores.get(k, 0) + s
    roots = [next(iter(h)) for h in mix]
    return dag.nodes, roots, picks


def volume_mixtures(vol_c: np.ndarray, nseg: int):
    """(mixtures, where): the distinct reduced count vectors of mip voxels of levels >= 1 with two
    or more segments, in scanline order of first appearance; where[(level, z, y, x)] = index."""
    nz, ny, nx = vol_c.shape
    mixtures, index, where = [], {}, {}
    for level in range(1, len(mipmap.level_dims((nx, ny, nz)))):
        c = mipmap.counts_level(vol_c, nseg, level)
        lz, ly, lx = c.shape[:3]
        for z in range(lz):
            for y in range(ly):
                for x in range(lx):
                    v = c[z, y, x]
                    nzs = np.nonzero(v)[0]
                    if len(nzs) < 2:
                        continue
                    g = 0
                    for s in nzs:
                        g = gcd(g, int(v[s]))
                    key = tuple((int(s), int(v[s]) // g) for s in nzs)
                    if key not in index:
                        index[key] = len(mixtures)
                        mixtures.append(dict(key))
                    where[(level, z, y, x)] = index[key]
    return mixtures, where
