"""CPU tests of the graph builder (mg_build) and the host side of the C ABI.

The builder's output is checked against the oracle: every mip voxel's node,
expanded exactly through the exported DAG (oracle.dag), must equal the
normalized histogram of that voxel's level-0 support (oracle.mipmap). That
pins the factorization as lossless (Sec. "Reconstruction": the graph
reconstructs the mipmap; with exact weights, without any loss).
"""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

from conftest import ROOT, golden
from oracle import dag, mipmap, scan
from paper_2009_02702_amd import Graph, MGError, SYMBOLS, synth
from paper_2009_02702_amd import _lib


def _exact_check(vol):
    g = Graph.build(vol)
    inf = g.info()
    S = inf["nseg"]
    d = g.export_dag()
    ids, vol_c = scan.compact(vol)
    assert np.array_equal(g.segment_ids(), ids.astype(np.uint32))
    mix = dag.expand_exact(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:], d["wden"][S:])
    assert len(mipmap.level_dims(vol.shape[::-1])) == inf["n_levels"]
    for l in range(inf["n_levels"]):
        m = g.export_map(l)
        c = mipmap.counts_level(vol_c, S, l)
        assert m.shape == c.shape[:3]
        for idx in np.ndindex(m.shape):
            cc = c[idx]
            tot = int(cc.sum())
            want = {s: Fraction(int(cc[s]), tot) for s in np.nonzero(cc)[0].tolist()}
            assert mix[int(m[idx])] == want, (l, idx)
    return g, d


def _invariants(g, d):
    inf = g.info()
    S, N = inf["nseg"], inf["n_nodes"]
    a, b = d["child_a"].astype(np.int64), d["child_b"].astype(np.int64)
    ids = np.arange(N)
    internal = ids >= S
    assert (a[internal] < ids[internal]).all() and (b[internal] < ids[internal]).all()   # children first
    assert (a[internal] != b[internal]).all()                                           # in-degree 2
    wn, wd = d["wnum"][internal].astype(object), d["wden"][internal].astype(object)
    assert all(0 < x and 2 * x <= y for x, y in zip(wn, wd))                             # w in (0, 1/2]
    assert np.array_equal(d["alpha"][internal], (d["wnum"][internal] / d["wden"][internal]).astype(np.float32))
    lv = dag.levels(S, a[S:], b[S:])
    assert np.array_equal(lv, d["rank"])
    assert inf["depth"] == (int(lv.max()) if N else 0)
    first, last = dag.defer_window(S, a[S:], b[S:])
    st = d["step"].astype(np.int64)
    assert (st[internal] >= first[internal]).all() and (st[internal] <= last[internal]).all()
    rp = d["rank_ptr"].astype(np.int64)
    assert rp[0] == 0 and rp[1] == S and rp[-1] == N
    for r in range(1, inf["depth"] + 1):
        assert (d["rank"][rp[r]:rp[r + 1]] == r).all()          # IDs sorted by rank
    sp = d["step_ptr"].astype(np.int64)
    sched = d["sched"].astype(np.int64)
    assert sp[0] == 0 and sp[1] == S and sp[-1] == N
    assert np.array_equal(np.sort(sched), np.arange(N))
    assert np.array_equal(sched[:S], np.arange(S))
    for s in range(1, inf["depth"] + 1):
        assert (st[sched[sp[s]:sp[s + 1]]] == s).all()


def _rand(shape, nseg, seed):
    return np.random.default_rng(seed).integers(0, nseg, size=shape).astype(np.uint32)


@pytest.mark.parametrize("shape,nseg,seed", [((7, 6, 5), 5, 0), ((8, 8, 8), 3, 1), ((3, 1, 9), 4, 2),
                                             ((1, 1, 1), 1, 3), ((5, 5, 5), 1, 4), ((2, 9, 4), 7, 5)])
def test_builder_lossless_random(shape, nseg, seed):
    g, d = _exact_check(_rand(shape, nseg, seed))
    _invariants(g, d)


def test_builder_lossless_voronoi_and_cylinders():
    vol = synth.make_volume(synth.workload(2, dims=(19, 17, 13), segments=9))
    g, d = _exact_check(vol)
    _invariants(g, d)
    vol = synth.make_volume(synth.workload(4, dims=(21, 15, 11), segments=12))
    g, d = _exact_check(vol)
    _invariants(g, d)
    vol = synth.make_volume(synth.workload(3, dims=(24, 20, 6), segments=10))
    g, d = _exact_check(vol)
    _invariants(g, d)


@pytest.mark.parametrize("config,dims,segments", [(2, (40, 36, 34), 30), (3, (64, 48, 16), 12),
                                                  (4, (33, 40, 36), 25)])
def test_rank1_and_rank2_nodes_on_full_cubes_split_into_whole_voxels(config, dims, segments):
    """The query kernels split a run of cubes on a rank-1 or rank-2 node into integer source
    counts when the node's fp32 weight times 8^level is a whole number k (the voxels on the b
    side), a rank-1 side of a rank-2 node splitting its n voxels per cube at the integer nearest
    n w' when that is within n 2^-22. For the exact graph this holds on every full cube (levels
    <= 7) whose node has rank 1 or 2, and the split is the cube's histogram: the node is the
    cube's own mixture."""
    vol = synth.make_volume(synth.workload(config, dims=dims, segments=segments))
    g = Graph.build(vol)
    inf = g.info()
    S = inf["nseg"]
    d = g.export_dag()
    r1_end, r2_end = int(d["rank_ptr"][2]), int(d["rank_ptr"][3])
    alpha = d["alpha"].astype(np.float32)
    _, vol_c = scan.compact(vol)
    X, Y, Z = dims
    seen = [0, 0]

    def side(hist, s, n):  # n voxels per cube on a side: a source, or a rank-1 node's split
        if n == 0:
            return
        if s < S:
            hist[s] += n
            return
        mf = np.float32(alpha[s] * np.float32(n))
        m = int(np.rint(mf))
        assert abs(float(mf) - m) <= n * 2.0 ** -22 and 0 <= m <= n
        hist[int(d["child_a"][s])] += n - m
        hist[int(d["child_b"][s])] += m

    for l in range(1, min(inf["n_levels"], 8)):
        m = g.export_map(l)
        c = mipmap.counts_level(vol_c, S, l)
        cube = 8 ** l
        for z in range(Z >> l):
            for y in range(Y >> l):
                for x in range(X >> l):
                    v = int(m[z, y, x])
                    if not S <= v < r2_end:
                        continue
                    k = np.float32(alpha[v] * np.float32(cube))
                    assert float(k) == int(k), (l, (x, y, z), v)
                    hist = np.zeros(S, dtype=np.int64)
                    side(hist, int(d["child_a"][v]), cube - int(k))
                    side(hist, int(d["child_b"][v]), int(k))
                    assert np.array_equal(hist, c[z, y, x].astype(np.int64)), (l, (x, y, z), v)
                    seen[v >= r1_end] += 1
    assert seen[0] > 0 and seen[1] > 0
    # a quantized graph's weights are not such fractions in general: the kernels push those
    q = g.quantize(5)
    qa = q.export_dag()["alpha"]
    m1 = g.export_map(1)
    on1 = [int(v) for v in np.unique(m1) if S <= v < r1_end]
    assert any(float(np.float32(qa[v]) * 8) != int(np.float32(qa[v]) * 8) for v in on1)


def test_builder_sparse_ids_and_uint16():
    vol = np.array([[[4000000000, 7, 7, 123456789], [7, 7, 5, 5]]], dtype=np.uint32)
    g, d = _exact_check(vol)
    assert g.segment_ids().tolist() == [5, 7, 123456789, 4000000000]
    v16 = _rand((4, 5, 6), 300, 9).astype(np.uint16) * 200
    g = Graph.build(v16)
    assert np.array_equal(g.segment_ids(), np.unique(v16).astype(np.uint32))


def test_builder_paper_mixtures():
    """The mixtures m and m' of Fig. 'DAG' as whole-volume histograms; pushing mass 1 from the
    top node through the exported DAG yields them (caption of Fig. 'DAG')."""
    fx = golden("dag_figure.json")
    for name in ("lambda7", "lambda9"):
        want = [Fraction(v) for v in fx["mixtures"][name]]
        vol = np.concatenate([np.full(int(v * 10), s, dtype=np.uint32) for s, v in enumerate(want)])
        vol = vol.reshape(1, 1, 10)
        g, d = _exact_check(vol)
        S = g.info()["nseg"]
        top = int(g.export_map(g.info()["n_levels"] - 1)[0, 0, 0])
        mass = np.zeros(g.info()["n_nodes"])
        mass[top] = 1.0
        got = dag.push(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:] / d["wden"][S:], mass)
        assert np.allclose(got, [float(v) for v in want], atol=1e-15)


def test_builder_canonical_orientation():
    """(i, j, w) == (j, i, 1-w) (Sec. 'Implementation Details'): stored with w <= 1/2, heavier part as a.
    Fig. 'factorization': lambda5 = 1/3 e1 + 2/3 e2 is stored as a = e2, b = e1, w = 1/3."""
    vol = np.array([[[0, 1, 1]]], dtype=np.uint32)
    g = Graph.build(vol)
    d = g.export_dag()
    top = int(g.export_map(g.info()["n_levels"] - 1)[0, 0, 0])
    assert (d["child_a"][top], d["child_b"][top], d["wnum"][top], d["wden"][top]) == (1, 0, 1, 3)


def test_builder_depth_cap_and_bad_args():
    vol = _rand((8, 8, 8), 40, 11)
    g = Graph.build(vol)
    depth = g.info()["depth"]
    assert depth == int(np.ceil(np.log2(g.info()["max_mixture"])))
    with pytest.raises(MGError) as e:
        Graph.build(vol, max_depth=depth - 1)
    assert e.value.code == -5
    with pytest.raises(ValueError):
        Graph.build(np.zeros((2, 2), dtype=np.uint32))
    with pytest.raises(ValueError):
        Graph.build(-np.ones((2, 2, 2), dtype=np.int32))
    with pytest.raises(MGError) as e:
        Graph.build(np.zeros((0, 2, 2), dtype=np.uint32))
    assert e.value.code == -1


def test_builder_deterministic_across_threads():
    vol = synth.make_volume(synth.workload(2, dims=(40, 36, 30), segments=30))
    a = Graph.build(vol, threads=1)
    b = Graph.build(vol, threads=7)
    da, db = a.export_dag(), b.export_dag()
    for k in da:
        assert np.array_equal(da[k], db[k]), k
    for l in range(a.info()["n_levels"]):
        assert np.array_equal(a.export_map(l), b.export_map(l))


def test_builder_no_defer_steps_are_ranks():
    vol = synth.make_volume(synth.workload(2, dims=(20, 20, 20), segments=20))
    g = Graph.build(vol, defer=False)
    d = g.export_dag()
    assert np.array_equal(d["step"], d["rank"])
    _invariants(g, d)


def test_defer_fills_steps():
    """Deferred scheduling (Sec. 'Reconstruction'): each step is filled to ceil(N/depth) nodes while
    deferrable nodes remain."""
    vol = synth.make_volume(synth.workload(2, dims=(48, 48, 48), segments=60))
    g = Graph.build(vol)
    d = g.export_dag()
    inf = g.info()
    S, N, D = inf["nseg"], inf["n_nodes"], inf["depth"]
    target = -(-(N - S) // D)
    sizes = np.diff(d["step_ptr"].astype(np.int64))[1:]
    first, last = dag.defer_window(S, d["child_a"][S:], d["child_b"][S:])
    st = d["step"].astype(np.int64)
    for s in range(1, D + 1):
        if sizes[s - 1] < target:
            # nothing that could still have run here was left for later
            later = (st > s) & (first <= s) & (np.arange(N) >= S)
            assert not later.any(), s


def test_save_load_roundtrip_and_corruption(tmp_path):
    vol = synth.make_volume(synth.workload(2, dims=(17, 18, 19), segments=11))
    g = Graph.build(vol)
    p = str(tmp_path / "g.mg")
    g.save(p)
    h = Graph.load(p)
    da, db = g.export_dag(), h.export_dag()
    for k in da:
        assert np.array_equal(da[k], db[k])
    for l in range(g.info()["n_levels"]):
        assert np.array_equal(g.export_map(l), h.export_map(l))
    raw = bytearray(open(p, "rb").read())
    raw[200] ^= 0x55
    q = str(tmp_path / "bad.mg")
    open(q, "wb").write(bytes(raw))
    with pytest.raises(MGError) as e:
        Graph.load(q)
    assert e.value.code in (-7, -6)
    with pytest.raises(MGError) as e:
        Graph.load(str(tmp_path / "missing.mg"))
    assert e.value.code == -6


def test_abi_exports_every_declared_symbol():
    src = open(os.path.join(ROOT, "include", "mg.h")).read()
    declared = sorted(set(re.findall(r"\b(mg_[a-z_]+)\s*\(", src)))
    assert sorted(SYMBOLS) == declared
    lib = _lib.load()
    for name in declared:
        assert hasattr(lib, name), name


def test_gpu_calls_before_upload_are_state_errors():
    g = Graph.build(_rand((4, 4, 4), 3, 12))
    lib = _lib.load()
    rc = lib.mg_query_boxes(g._h, 1, 1, 1, 1, 1, None)
    assert rc == -4
    rc = lib.mg_propagate_tf(g._h, 1, 1, 1, None)
    assert rc == -4
    assert b"mg_upload" in lib.mg_last_error()
    # n = 0 is a no-op even without a device
    assert lib.mg_query_boxes(g._h, None, 0, None, None, 0, None) == 0


def test_mixture_lut_rows_are_the_exact_mixtures():
    """mg_lut_build (Sec. 'Decoder', mixture lookup): row n lists exactly the segments of node n's
    mixture, each fraction within one fp32 unit of the exact rational value (oracle.dag.expand_exact),
    sources in increasing order."""
    for w in (synth.workload(2, dims=(19, 17, 13), segments=9), synth.workload(4, dims=(21, 15, 11), segments=12)):
        g = Graph.build(synth.make_volume(w))
        S, N = g.info()["nseg"], g.info()["n_nodes"]
        nnz = g.lut_build(threads=3)
        ptr, seg, val = g.export_lut()
        assert ptr[0] == 0 and int(ptr[-1]) == nnz == len(seg) and np.all(np.diff(ptr.astype(np.int64)) >= 1)
        d = g.export_dag()
        mix = dag.expand_exact(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:], d["wden"][S:])
        for n in range(N):
            row = slice(int(ptr[n]), int(ptr[n + 1]))
            s_row, v_row = seg[row].tolist(), val[row]
            assert s_row == sorted(mix[n]), n
            want = np.array([float(mix[n][s]) for s in s_row], dtype=np.float64)
            ulp = np.spacing(want.astype(np.float32)).astype(np.float64)
            assert np.all(np.abs(v_row.astype(np.float64) - want) <= ulp), n


def test_mixture_lut_threads_deterministic_and_state_errors():
    g = Graph.build(_rand((9, 8, 7), 6, 21))
    with pytest.raises(MGError) as e:
        g.export_lut()
    assert e.value.code == -4
    g.lut_build(threads=1)
    a = g.export_lut()
    g.lut_build(threads=8)
    b = g.export_lut()
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_server_cube_counts_match_the_oracle():
    """The server's closed-form cube count per box (size-aware admission) equals the footprint's cube
    count of the oracle (Alg. footprint assembly), clipped boxes and empty boxes included."""
    from oracle import footprint as ofp
    from paper_2009_02702_amd.serve import cube_counts
    rng = np.random.default_rng(3)
    dims = (37, 23, 50)
    b = np.concatenate([rng.integers(0, 45, (300, 3)), rng.integers(0, 40, (300, 3))], axis=1).astype(np.uint32)
    b[:5, 3:] = 0
    got = cube_counts(b, dims)
    for i, row in enumerate(b.astype(int)):
        assert got[i] == ofp.cube_count(row[:3], row[3:], dims), i


def test_server_split_box_tiles_the_box_at_aligned_cuts():
    from paper_2009_02702_amd.serve import split_box
    rng = np.random.default_rng(4)
    dims = (300, 200, 250)
    for _ in range(200):
        box = np.concatenate([rng.integers(0, 290, 3), rng.integers(1, 300, 3)]).astype(np.uint32)
        p = int(rng.integers(1, 40))
        sub = split_box(box, dims, p).astype(np.int64)
        lo = np.minimum(box[:3].astype(np.int64), dims)
        hi = np.minimum(box[:3].astype(np.int64) + box[3:], dims)
        assert np.prod(sub[:, 3:], axis=1).sum() == np.prod(np.maximum(hi - lo, 0))
        assert (sub[:, 3:] > 0).all() or len(sub) == 1
        ax = int(np.argmax(hi - lo))
        inner = sub[1:, ax]                                  # cut positions share one power of two
        if len(inner):
            step = inner[1] - inner[0] if len(inner) > 1 else None
            assert step is None or (step & (step - 1)) == 0
            assert (inner % (step or 1) == 0).all()


def test_server_admission_step():
    """One admission step of the server (host logic, no GPU): requests are taken from the head of
    the queue while their rows fit max_batch and at most max_tf carry a transfer function; the
    head is never skipped, so the queue order is kept."""
    from collections import deque

    from paper_2009_02702_amd.serve import Server
    srv = Server.__new__(Server)
    srv.max_batch, srv.max_tf = 4, 1
    rows = {2: [0, 1, 2]}                 # request 2 was split into three sub-boxes
    ti = np.array([-1, 0, -1, 1, -1, -1])
    q = deque(range(6))
    take, n_rows, n_tf = srv._admit(q, rows, ti)
    assert take == [0, 1] and n_rows == 2 and n_tf == 1     # request 2's 3 rows would exceed 4
    take, n_rows, n_tf = srv._admit(q, rows, ti)
    assert take == [2, 3] and n_rows == 4 and n_tf == 1     # full: 3 + 1 rows
    srv.max_batch = 8
    q = deque([3, 1, 4])
    take, n_rows, n_tf = srv._admit(q, rows, ti)
    assert take == [3] and n_tf == 1                        # a second TF request waits for the next batch
    take, n_rows, n_tf = srv._admit(q, rows, ti)
    assert take == [1, 4] and n_tf == 1
    assert not q
    take, n_rows, n_tf = srv._admit(q, rows, None)
    assert take == [] and n_rows == 0
