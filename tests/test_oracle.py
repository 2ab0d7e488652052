"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU. None compares the oracle with itself: the
checks are the paper's worked examples and printed tables (tests/golden/),
library routines for special cases (numpy.bincount), brute-force
enumeration on tiny inputs, closed forms and invariants.
"""
import itertools
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

from conftest import golden
from oracle import dag, footprint, mipmap, scan, tf


def _rand_vol(shape, nseg, seed):
    g = np.random.default_rng(seed)
    return g.integers(0, nseg, size=shape).astype(np.uint32)


def _blocky_vol(shape, nseg, seed, block=3):
    """Random piecewise-constant labels (so that mip voxels are often pure)."""
    g = np.random.default_rng(seed)
    nz, ny, nx = shape
    coarse = g.integers(0, nseg, size=((nz + block - 1) // block, (ny + block - 1) // block, (nx + block - 1) // block))
    vol = np.repeat(np.repeat(np.repeat(coarse, block, 0), block, 1), block, 2)[:nz, :ny, :nx]
    return np.ascontiguousarray(vol.astype(np.uint32))


# ------------------------------------------------------------------ O1 (brute-force scan)

def test_o1_all_boxes_tiny_volume_vs_bincount():
    """Exhaustive: every box of a 5x6x7 volume equals numpy.bincount of the slice."""
    vol = _rand_vol((7, 6, 5), 4, 1)
    nz, ny, nx = vol.shape
    boxes = []
    for x0, x1 in itertools.combinations(range(nx + 1), 2):
        for y0, y1 in itertools.combinations(range(ny + 1), 2):
            for z0, z1 in itertools.combinations(range(nz + 1), 2):
                boxes.append((x0, y0, z0, x1 - x0, y1 - y0, z1 - z0))
    boxes = np.array(boxes, dtype=np.uint32)
    counts, pr = scan.box_counts(vol, 4, boxes, threads=4)
    for q in range(0, len(boxes), 7):
        ref = scan.box_counts_numpy(vol, 4, boxes[q])
        assert np.array_equal(counts[q], ref)
    vols = boxes[:, 3:].astype(np.int64).prod(axis=1)
    assert np.array_equal(counts.sum(axis=1).astype(np.int64), vols)          # mass = box volume
    assert np.allclose(pr.sum(axis=1), 1.0, rtol=0, atol=1e-12)                # convex (Eq. convex1)
    assert (pr >= 0).all()                                                     # Eq. convex2


def test_o1_single_voxel_is_one_hot_and_full_box_is_global_histogram():
    vol = _rand_vol((9, 8, 11), 6, 2)
    nz, ny, nx = vol.shape
    g = np.random.default_rng(3)
    pts = g.integers(0, [nx, ny, nz], size=(50, 3))
    boxes = np.concatenate([pts, np.ones_like(pts)], axis=1).astype(np.uint32)
    counts, pr = scan.box_counts(vol, 6, boxes)
    for q, (x, y, z) in enumerate(pts):
        assert pr[q].tolist() == [1.0 if s == vol[z, y, x] else 0.0 for s in range(6)]
    full = np.array([[0, 0, 0, nx, ny, nz]], dtype=np.uint32)
    c, p = scan.box_counts(vol, 6, full)
    assert np.array_equal(c[0], np.bincount(vol.ravel(), minlength=6).astype(np.uint64))


def test_o1_clipping_and_empty_boxes():
    vol = _rand_vol((4, 5, 6), 3, 4)
    nz, ny, nx = vol.shape
    boxes = np.array([
        [4, 3, 2, 100, 100, 100],   # clipped to the volume
        [6, 0, 0, 2, 2, 2],         # origin at the x extent: empty
        [0, 0, 0, 0, 3, 3],         # zero extent: empty
        [0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF],   # huge extents clip, no overflow
    ], dtype=np.uint32)
    counts, pr = scan.box_counts(vol, 3, boxes)
    ref0 = np.bincount(vol[2:, 3:, 4:].ravel(), minlength=3)
    assert np.array_equal(counts[0], ref0.astype(np.uint64))
    assert counts[1].sum() == 0 and (pr[1] == 0).all()
    assert counts[2].sum() == 0 and (pr[2] == 0).all()
    assert counts[3].sum() == nx * ny * nz


def test_o1_paper_mixtures():
    """Volumes whose histograms are the paper's m and m' (caption of Fig. 'DAG')."""
    fx = golden("dag_figure.json")
    for name in ("lambda7", "lambda9"):
        want = [Fraction(v) for v in fx["mixtures"][name]]
        cnt = [int(v * 10) for v in want]
        vol = np.concatenate([np.full(c, s, dtype=np.uint32) for s, c in enumerate(cnt)])
        vol = np.random.default_rng(0).permutation(vol).reshape(1, 2, 5)
        c, p = scan.box_counts(vol, 4, np.array([[0, 0, 0, 5, 2, 1]], dtype=np.uint32))
        assert [Fraction(float(v)).limit_denominator(100) for v in p[0]] == want


def test_o1_compaction_keeps_id_order():
    vol = np.array([[[900, 7, 7, 65000]]], dtype=np.uint32)
    ids, counts, pr = scan.box_histogram(vol, np.array([[0, 0, 0, 4, 1, 1]], dtype=np.uint32))
    assert ids.tolist() == [7, 900, 65000]
    assert counts[0].tolist() == [2, 1, 1]


def test_o1_compaction_table_path_equals_numpy_unique():
    """The linear-time compaction (IDs below 2^28) gives what numpy.unique gives; IDs of 2^28 and
    above take numpy.unique itself."""
    rng = np.random.default_rng(3)
    for hi in (5, 1000, (1 << 28) - 1, 1 << 31):
        vol = rng.integers(0, hi, size=(7, 9, 11), dtype=np.uint64).astype(np.uint32)
        vol[0, 0, 0] = hi - 1
        ids, vc = scan.compact(vol)
        u, inv = np.unique(vol.ravel(), return_inverse=True)
        assert ids.tolist() == u.tolist()
        assert np.array_equal(vc.ravel(), inv.astype(np.uint32))
        assert vc.shape == vol.shape and vc.dtype == np.uint32


# ------------------------------------------------------------------ footprint assembly

def test_footprint_paper_figure_2d():
    fx = golden("footprint_figure.json")
    (x0, y0), (dx, dy), (nx, ny) = fx["origin"], fx["extent"], fx["dims"]
    assert [list(s) for s in footprint.footprint_1d(x0, dx, nx)] == fx["steps_x"]
    assert [list(s) for s in footprint.footprint_1d(y0, dy, ny)] == fx["steps_y"]
    cubes = footprint.assembly((x0, y0), (dx, dy), (nx, ny))
    lv = Counter(l for l, _ in cubes)
    assert {str(k): v for k, v in lv.items()} == fx["squares_per_level"]
    assert len(cubes) == fx["squares_total"]
    assert sum(4 ** l for l, _ in cubes) == fx["voxels"]                  # 2D: 4^l voxels per square
    assert sorted(cubes) == sorted(footprint.maximal_cubes((x0, y0), (dx, dy), (nx, ny)))


def test_footprint_equals_maximal_cubes_3d_random():
    g = np.random.default_rng(5)
    dims = (37, 29, 41)
    for _ in range(400):
        p = g.integers(0, 45, size=3)
        dp = g.integers(0, 30, size=3)
        a = sorted(footprint.assembly(p, dp, dims))
        b = sorted(footprint.maximal_cubes(p, dp, dims))
        assert a == b
        lo = [min(int(p[i]), dims[i]) for i in range(3)]
        hi = [min(int(p[i]) + int(dp[i]), dims[i]) for i in range(3)]
        vol = int(np.prod([max(0, h - l) for l, h in zip(lo, hi)]))
        assert sum(8 ** l for l, _ in a) == vol                              # Sigma 8^l = |box|
        assert len(set(a)) == len(a)
        assert footprint.cube_count(p, dp, dims) == len(a)


def test_footprint_cubes_tile_the_box_exactly():
    dims = (16, 16, 16)
    p, dp = (3, 1, 5), (11, 14, 9)
    cover = np.zeros((16, 16, 16), dtype=np.int32)
    for l, c in footprint.assembly(p, dp, dims):
        s = 1 << l
        cover[c[2] * s:(c[2] + 1) * s, c[1] * s:(c[1] + 1) * s, c[0] * s:(c[0] + 1) * s] += 1
    want = np.zeros_like(cover)
    want[5:14, 1:15, 3:14] = 1
    assert np.array_equal(cover, want)


def test_footprint_fetch_counts_match_table_query():
    """Statistical pin: mean cube count of randomly aligned e^3 boxes vs the paper's fetch column."""
    fx = golden("table_query.json")
    for k, e in enumerate(fx["edges"]):
        paper = [fx["fetches"][d][k] for d in ("hippocampus", "neocortex", "polymer")]
        ours = footprint.expected_cube_count(e, samples=600, seed=11 + k)
        assert abs(ours - np.mean(paper)) / np.mean(paper) < 0.10, (e, ours, paper)
        # each dataset's printed fetch count, within the scatter of a small sample
        for v in paper:
            assert abs(ours - v) / v < 0.30


def test_table_query_saved_is_one_minus_fetches_over_voxels():
    """The table's 'saved' column is 1 - fetches / e^3: one fetch is one cube sample."""
    fx = golden("table_query.json")
    for d in fx["fetches"]:
        for e, f, s in zip(fx["edges"], fx["fetches"][d], fx["saved_percent"][d]):
            assert abs(100 * (1 - f / e ** 3) - s) < 0.35, (d, e, f, s)


# ------------------------------------------------------------------ mipmap

def test_mipmap_levels_and_voxels_match_table_factorization():
    fx = golden("table_factorization.json")
    for v in fx["volumes"]:
        dims = v["dims"]
        assert len(mipmap.level_dims(dims)) == v["levels"]
        tot = mipmap.total_voxels(dims) / 1e6
        assert abs(tot - v["voxels_million"]) / v["voxels_million"] < 0.001, (v["name"], tot)


def test_mipmap_convex_level0_unit_and_top_is_global_histogram():
    vol = _rand_vol((5, 7, 6), 5, 6)
    nz, ny, nx = vol.shape
    nlev = len(mipmap.level_dims((nx, ny, nz)))
    h0 = mipmap.mixtures_level(vol, 5, 0)
    assert np.array_equal(h0.argmax(-1), vol) and np.array_equal(h0.max(-1), np.ones_like(h0.max(-1)))
    for l in range(nlev):
        for mode in ("voxels", "children"):
            h = mipmap.mixtures_level(vol, 5, l, mode)
            assert np.allclose(h.sum(-1), 1.0, atol=1e-12) and (h >= 0).all()
    top = mipmap.mixtures_level(vol, 5, nlev - 1)
    assert top.shape[:3] == (1, 1, 1)
    assert np.allclose(top[0, 0, 0], np.bincount(vol.ravel(), minlength=5) / vol.size, atol=1e-15)


def test_mipmap_modes_agree_on_power_of_two_and_differ_at_borders():
    vol = _rand_vol((8, 8, 8), 3, 7)
    for l in range(4):
        assert np.allclose(mipmap.mixtures_level(vol, 3, l, "voxels"), mipmap.mixtures_level(vol, 3, l, "children"))
    vol = np.zeros((1, 1, 3), dtype=np.uint32)
    vol[0, 0, 2] = 1
    # level 2 of a 3-voxel row: voxel weights give 1/3, child averaging gives 1/2 (children 2 and 1 voxels)
    assert np.allclose(mipmap.mixtures_level(vol, 2, 2, "voxels")[0, 0, 0], [2 / 3, 1 / 3])
    assert np.allclose(mipmap.mixtures_level(vol, 2, 2, "children")[0, 0, 0], [1 / 2, 1 / 2])


def test_footprint_query_from_mipmap_equals_o1():
    """Eq. (mip) + footprint assembly, denormalised by 8^l, reproduce the brute-force counts exactly."""
    vol = _blocky_vol((13, 11, 9), 5, 8)
    nz, ny, nx = vol.shape
    nlev = len(mipmap.level_dims((nx, ny, nz)))
    counts = [mipmap.counts_level(vol, 5, l) for l in range(nlev)]
    g = np.random.default_rng(9)
    boxes = np.concatenate([g.integers(0, [nx, ny, nz], size=(150, 3)), g.integers(0, 12, size=(150, 3))], 1)
    boxes = boxes.astype(np.uint32)
    o1 = scan.box_counts(vol, 5, boxes, probs=False)
    for q, b in enumerate(boxes):
        acc = np.zeros(5, dtype=np.int64)
        for l, (cx, cy, cz) in footprint.assembly(b[:3], b[3:], (nx, ny, nz)):
            h = counts[l][cz, cy, cx]
            assert h.sum() == 8 ** l                     # every cube is a full, interior cube
            acc += h
        assert np.array_equal(acc.astype(np.uint64), o1[q])


# ------------------------------------------------------------------ transfer functions

def test_tf_constant_and_one_hot():
    vol = _rand_vol((6, 5, 7), 4, 10)
    nz, ny, nx = vol.shape
    const = np.tile(np.array([[10, 20, 30, 40]], dtype=np.uint8), (4, 1))
    for l in range(len(mipmap.level_dims((nx, ny, nz)))):
        c = tf.level_colours(vol, 4, const, l)
        assert np.allclose(c, np.array([10, 20, 30, 40]) / 255.0, atol=1e-15)
    onehot = np.zeros((4, 4), dtype=np.uint8)
    onehot[2, 0] = 255
    for l in range(3):
        c = tf.level_colours(vol, 4, onehot, l)
        h = mipmap.mixtures_level(vol, 4, l)
        assert np.allclose(c[..., 0], h[..., 2], atol=1e-15)
        assert np.allclose(c[..., 1:], 0.0)


def test_tf_voxel_colour_matches_level_colours():
    vol = _rand_vol((5, 9, 7), 6, 12)
    nz, ny, nx = vol.shape
    t = np.random.default_rng(13).integers(0, 256, size=(6, 4), dtype=np.uint8)
    for l in range(4):
        c = tf.level_colours(vol, 6, t, l)
        lz, ly, lx = c.shape[:3]
        for v in [(0, 0, 0), (lx - 1, ly - 1, lz - 1), (lx // 2, ly // 2, lz // 2)]:
            assert np.allclose(tf.voxel_colour(vol, t, l, v), c[v[2], v[1], v[0]], atol=1e-13)


# ------------------------------------------------------------------ DAG semantics

def _paper_dag():
    fx = golden("dag_figure.json")
    a = [n["a"] for n in fx["nodes"]]
    b = [n["b"] for n in fx["nodes"]]
    w = [Fraction(n["w"]) for n in fx["nodes"]]
    return fx, a, b, w


def test_dag_paper_example_exact():
    fx, a, b, w = _paper_dag()
    mix = dag.expand_exact(4, a, b, [x.numerator for x in w], [x.denominator for x in w])
    names = [n["name"] for n in fx["nodes"]]
    for name, want in fx["mixtures"].items():
        got = mix[4 + names.index(name)]
        assert [got.get(s, Fraction(0)) for s in range(4)] == [Fraction(v) for v in want]
    lv = dag.levels(4, a, b)
    assert {n: int(lv[4 + i]) for i, n in enumerate(names)} == fx["levels"]


def test_dag_push_paper_example_and_conservation():
    fx, a, b, w = _paper_dag()
    wf = [float(x) for x in w]
    names = [n["name"] for n in fx["nodes"]]
    for name in ("lambda7", "lambda9"):
        mass = np.zeros(9)
        mass[4 + names.index(name)] = 1.0
        got = dag.push(4, a, b, wf, mass)
        assert np.allclose(got, [float(Fraction(v)) for v in fx["mixtures"][name]], atol=1e-15)
    mass = np.random.default_rng(14).random(9) * 100
    assert abs(dag.push(4, a, b, wf, mass).sum() - mass.sum()) < 1e-10


def test_dag_adjoint_identity():
    """<push(c), t> = <c, forward(t)>: the push is the transpose of the forward propagation."""
    fx, a, b, w = _paper_dag()
    wf = [float(x) for x in w]
    g = np.random.default_rng(15)
    for _ in range(20):
        c = g.random(9)
        t = g.random(4)
        lhs = dag.push(4, a, b, wf, c) @ t
        rhs = c @ dag.forward(4, a, b, wf, t)
        assert abs(lhs - rhs) < 1e-12


def test_dag_levels_and_deferral_window_figure():
    fx = golden("dagtopo_figure.json")
    a = [n[0] for n in fx["nodes"]]
    b = [n[1] for n in fx["nodes"]]
    lv, last = dag.defer_window(fx["nseg"], a, b)
    assert lv.tolist() == fx["levels"]
    d = fx["deferrable"]
    assert (int(lv[d["node"]]), int(last[d["node"]])) == (d["first"], d["last"])
    # every other internal node has a window of one step
    for n in range(fx["nseg"], len(lv)):
        if n != d["node"] and n != len(lv) - 1:
            assert lv[n] == last[n]


def test_dag_rejects_cycles_and_bad_ids():
    with pytest.raises(ValueError):
        dag.levels(2, [0, 3], [1, 0])      # node 2 -> 3 -> 2 ... (3 uses 0 and 3)
    with pytest.raises(ValueError):
        dag.levels(2, [0], [5])
