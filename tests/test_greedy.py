"""The paper's greedy factorizer (Sec. "Compression", Eqs. greedy1 / greedy2; Sec. "Implementation
Details", cutoff tau): the oracle (oracle/greedy.py) pinned to hand-computed scores and picks and
to exact expansion, and the library's mg_build(factorizer=...) equal to the oracle node for node.
"""
from fractions import Fraction
import random

import numpy as np
import pytest

from oracle import dag as odag
from oracle import greedy, scan
from paper_2009_02702_amd import Graph, synth


# Fig. "DAG": m = (0.1, 0.2, 0.3, 0.4) and m' = (0.2, 0.4, 0.1, 0.3), as voxel counts
FIG_M = {0: 1, 1: 2, 2: 3, 3: 4}
FIG_M2 = {0: 2, 1: 4, 2: 1, 3: 3}


def test_scores_by_hand():
    s1 = greedy.phi([FIG_M, FIG_M2], "occurrence")
    s2 = greedy.phi([FIG_M, FIG_M2], "reduction")
    # both mixtures hold every pair: phi1 = 2; four components each: phi2 = 2 x (4 - 1)
    assert s1 == {k: 2 for k in [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]}
    assert s2 == {k: 6 for k in s1}
    # a mixture of two components adds 2 to its pair under phi2, one of three adds 3 - 1 = 2
    assert greedy.phi([{5: 1, 7: 3}], "reduction") == {(5, 7): 2}
    assert greedy.phi([{5: 1, 7: 3, 9: 1}], "reduction") == {(5, 7): 2, (5, 9): 2, (7, 9): 2}


def test_equal_ratios_share_a_node_as_in_the_figure():
    """All pairs tie, so the first pick is (e_0, e_1); both mixtures hold them in the ratio 1:2 and
    share one node, 2/3 e_1 + 1/3 e_0 (Fig. "DAG": lambda_5 is re-used by m and m')."""
    nodes, roots, picks = greedy.factorize(4, [FIG_M, FIG_M2], "reduction", tau=0)
    assert picks[0] == (0, 1)
    assert nodes[0] == (1, 0, 1, 3)
    # no other node mixes e_0 and e_1 directly, and both mixtures were factored through node 4
    assert sum(1 for nd in nodes if nd[:2] in ((0, 1), (1, 0))) == 1
    def reaches(n, target):
        return n == target or (n >= 4 and any(reaches(c, target) for c in nodes[n - 4][:2]))
    assert len(roots) == 2 and all(reaches(r, 4) for r in roots)


def test_strategies_pick_differently():
    """A = B = {e0, e1} and C with six segments: phi1(0, 1) = 2 beats phi1 = 1 of C's pairs; phi2
    gives C's pairs 6 - 1 = 5 and (0, 1) only 2 + 2 = 4."""
    A = {0: 1, 1: 1}
    C = {s: 1 for s in range(2, 8)}
    _, _, p1 = greedy.factorize(8, [A, dict(A), C], "occurrence", tau=0)
    _, _, p2 = greedy.factorize(8, [A, dict(A), C], "reduction", tau=0)
    assert p1[0] == (0, 1)
    assert p2[0] == (2, 3)


def test_cutoff_keeps_small_mixtures_out_of_the_global_search():
    """With tau = 3 a three-segment mixture never takes part in stage 1: its pairs are not picked
    there, however often they occur."""
    small = [{0: 1, 1: 2, 2: 3} for _ in range(5)]
    big = {s: s + 1 for s in range(3, 8)}
    _, _, picks = greedy.factorize(8, small + [big], "occurrence", tau=3)
    assert all(i >= 3 and j >= 3 for i, j in picks) and len(picks) == 2   # 5 segments -> 3
    _, _, picks0 = greedy.factorize(8, small + [big], "occurrence", tau=0)
    assert picks0[0] == (0, 1)


@pytest.mark.parametrize("strategy,tau", [("reduction", 0), ("reduction", 3), ("occurrence", 3), ("occurrence", 1)])
def test_every_root_expands_to_its_mixture(strategy, tau):
    """Brute force: each mixture's node, expanded exactly, is the normalized input mixture; the node
    count is between the largest mixture's n - 1 and the sum of n - 1."""
    rng = random.Random(7)
    S = 9
    mixes = []
    for _ in range(40):
        k = rng.randint(2, 7)
        segs = rng.sample(range(S), k)
        mixes.append({s: rng.choice([1, 1, 2, 3, 6]) for s in segs})
    nodes, roots, _ = greedy.factorize(S, mixes, strategy, tau)
    a = [n[0] for n in nodes]
    b = [n[1] for n in nodes]
    ex = odag.expand_exact(S, a, b, [n[2] for n in nodes], [n[3] for n in nodes])
    for h, r in zip(mixes, roots):
        tot = sum(h.values())
        assert ex[r] == {s: Fraction(c, tot) for s, c in h.items()}
    assert max(len(h) for h in mixes) - 1 <= len(nodes) <= sum(len(h) - 1 for h in mixes)
    for (na, nb, wn, wd) in nodes:
        assert 0 < wn and 2 * wn <= wd


def _canon(nseg, a, b, wn, wd, intern):
    """Canonical ID of every node: sources by index, others by (canon(a), canon(b), w)."""
    out = []
    for n in range(len(a)):
        key = ("s", n) if n < nseg else (out[a[n]], out[b[n]], int(wn[n]), int(wd[n]))
        out.append(intern.setdefault(key, len(intern)))
    return out


@pytest.mark.parametrize("config,dims,segments", [(1, (20, 18, 16), 8), (2, (26, 22, 20), 20), (4, (24, 20, 18), 12)])
@pytest.mark.parametrize("strategy,tau", [("reduction", 3), ("occurrence", 3), ("reduction", 0)])
def test_library_greedy_graph_equals_the_oracle(config, dims, segments, strategy, tau):
    w = synth.workload(config, dims=dims, segments=segments)
    vol = synth.make_volume(w)
    g = Graph.build(vol, factorizer=strategy, tau=tau)
    ids, vol_c = scan.compact(vol)
    S = len(ids)
    mixtures, where = greedy.volume_mixtures(vol_c, S)
    nodes, roots, _ = greedy.factorize(S, mixtures, strategy, tau)
    intern = {}
    oc = _canon(S, list(range(S)) + [n[0] for n in nodes], list(range(S)) + [n[1] for n in nodes],
                [0] * S + [n[2] for n in nodes], [1] * S + [n[3] for n in nodes], intern)
    d = g.export_dag()
    lc = _canon(S, d["child_a"], d["child_b"], d["wnum"], d["wden"], intern)
    assert g.info()["n_nodes"] == S + len(nodes)
    assert sorted(lc) == sorted(oc)
    for l in range(1, g.info()["n_levels"]):
        m = g.export_map(l)
        for (lev, z, y, x), k in where.items():
            if lev == l:
                assert lc[int(m[z, y, x])] == oc[roots[k]], (l, z, y, x)


def test_greedy_build_options():
    vol = synth.make_volume(synth.workload(1, dims=(12, 10, 8), segments=5))
    with pytest.raises(KeyError):
        Graph.build(vol, factorizer="exhaustive")
    import ctypes
    from paper_2009_02702_amd import _lib
    v = np.ascontiguousarray(vol.astype(np.uint32))
    o = _lib.BuildOpts(nx=v.shape[2], ny=v.shape[1], nz=v.shape[0], defer=1, factorizer=3)
    h = ctypes.c_void_p()
    assert _lib.load().mg_build(v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o), ctypes.byref(h)) == -1
    a = Graph.build(vol, factorizer="reduction", tau=3)
    b = Graph.build(vol, factorizer="reduction", tau=3, threads=1)
    assert a.info()["n_nodes"] == b.info()["n_nodes"]
    for k in ("child_a", "child_b", "wnum", "wden"):
        assert np.array_equal(a.export_dag()[k], b.export_dag()[k])


@pytest.mark.parametrize("factorizer", ["halving", "reduction", "occurrence"])
def test_degenerate_volumes_build_quantize_and_round_trip(factorizer):
    """One voxel, one segment, two alternating segments, a thin random column: every factorizer
    builds them; quantized copies survive the bit-packed stream."""
    vols = [np.array([[[7]]], dtype=np.uint32), np.full((4, 4, 4), 5, dtype=np.uint32),
            (np.arange(105).reshape(3, 5, 7) % 2).astype(np.uint32),
            np.random.default_rng(1).integers(0, 5, size=(9, 1, 1)).astype(np.uint32)]
    for vol in vols:
        for tau in (0, 3, 100):
            g = Graph.build(vol, factorizer=factorizer, tau=tau)
            ids, vol_c = scan.compact(vol)
            assert g.info()["nseg"] == len(ids)
            q = g.quantize(4)
            u = Graph.unpack(q.pack())
            assert u.info()["n_nodes"] == q.info()["n_nodes"] and u.pack() == q.pack()
