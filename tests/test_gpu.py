"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerance (no precision is fixed by the paper; derivation): counts from cubes
whose node is a source are exact integers; mass pushed through the DAG
carries, per hop, the fp32 rounding of the weight, of 1 - w and of the
product (3 units of 2^-24), and the compensated accumulation adds at most
about one unit per node; the graph depth here is ceil(log2 S) <= 14, so the
relative error per segment is below (5 * 14 + 2) * 2^-24 = 4.3e-6 < 1e-5.
Segments absent from a box must come out exactly 0, and boxes whose cubes are
all level-0 voxels must match the fp32-rounded oracle bit for bit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import footprint as ofp
from oracle import mipmap, scan
from oracle import tf as otf
from paper_2009_02702_amd import Graph, MGError, synth

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _compare(got, ref, level0_only=None, tag=""):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape, tag
    assert np.isfinite(got).all(), tag
    assert np.array_equal(got == 0, ref == 0), "%s: support differs" % tag
    nz = ref > 0
    rel = np.abs(got[nz] - ref[nz]) / ref[nz]
    assert rel.max(initial=0) <= REL_TOL, "%s: max rel err %g" % (tag, rel.max())
    if level0_only is not None and level0_only.any():
        a = got[level0_only].astype(np.float32)
        b = ref[level0_only].astype(np.float32)
        assert np.array_equal(a, b), "%s: level-0 boxes not bit-exact" % tag
    return rel.max(initial=0)


def _level0_only(g, dboxes):
    counts, _ = g.footprint(dboxes)
    c = counts.cpu().numpy()
    return (c[:, 1:].sum(axis=1) == 0) & (c[:, 0] > 0)


_GRAPHS = {}


def _graph(key, vol):
    if key not in _GRAPHS:
        _GRAPHS[key] = Graph.build(vol).upload(0)
    return _GRAPHS[key]


_LUT = set()


def _lut(g):
    """Build the mixture lookup table of a cached graph once."""
    if id(g) not in _LUT:
        g.lut_build()
        _LUT.add(id(g))
    return g


def _check_workload(w, n=None, variants=("batched", "plain", "naive"), key=None):
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w, n)
    g = _graph(key or (w.config, w.dims, w.segments), vol)
    if "lut" in variants:
        _lut(g)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    errs = {}
    for v in variants:
        out = g.query(db, variant=v)
        torch.cuda.synchronize()
        errs[v] = _compare(out.cpu().numpy(), ref, l0, "%s/%s" % (w.name, v))
    return g, errs


# ------------------------------------------------------------------ footprint (a1-a4)

def test_footprint_cubes_and_nodes_match_oracle():
    g0 = np.random.default_rng(21)
    vol = g0.integers(0, 6, size=(41, 29, 37)).astype(np.uint32)
    g = _graph("fp", vol)
    nx, ny, nz = 37, 29, 41
    boxes = np.concatenate([g0.integers(0, 45, size=(300, 3)), g0.integers(0, 40, size=(300, 3))], 1)
    boxes[:20, 3:] = 1
    boxes[20:30, :3] = 0
    boxes[20:30, 3:] = [nx, ny, nz]
    boxes = boxes.astype(np.uint32)
    counts, cubes = g.footprint(_dev(boxes), cubes_cap=2_000_000)
    counts = counts.cpu().numpy()
    cubes = cubes.cpu().numpy().astype(np.int64)
    maps = [g.export_map(l) for l in range(g.info()["n_levels"])]
    by_box = {}
    for q, l, x, y, z, node in cubes:
        by_box.setdefault(int(q), []).append((int(l), (int(x), int(y), int(z))))
        assert node == maps[l][z, y, x]
    for q, b in enumerate(boxes):
        want = sorted(ofp.assembly(b[:3], b[3:], (nx, ny, nz)))
        assert sorted(by_box.get(q, [])) == want, q
        hist = np.bincount([l for l, _ in want], minlength=len(maps)) if want else np.zeros(len(maps))
        assert np.array_equal(counts[q], hist), q


# ------------------------------------------------------------------ query parity (a1-a7, a10)

def test_query_config1_full():
    _, errs = _check_workload(synth.workload(1))
    print(errs)


@pytest.mark.parametrize("config,dims,segments,n", [
    (2, (96, 80, 72), 353, 3000),
    (3, (256, 256, 40), 1182, 2000),
    (4, (123, 96, 100), 1500, 3000),
    (5, (118, 113, 79), 353, 3000),
])
def test_query_reduced_recipes(config, dims, segments, n):
    _, errs = _check_workload(synth.workload(config, dims=dims, segments=segments, n_boxes=n))
    print(errs)


@pytest.mark.parametrize("config,dims,segments,n", [
    (2, (160, 150, 140), 300, 1500), (3, (256, 200, 40), 120, 800), (4, (150, 180, 120), 900, 800),
    (5, (118, 113, 79), 353, 800), (4, (160, 200, 150), 4000, 600),
])
def test_query_from_row_runs_every_row_length(config, dims, segments, n):
    """Slabs summed from row runs: runs for rows of every length (run_min_row 1), the default
    (rows of 16 cubes or more) and never (every slab streams cube by cube) all give the oracle's
    histograms, for the batched, plain and lookup-table queries and the sparse output; tiny tables
    send boxes through the retry and global-table launches with runs on. The last recipe has more
    sources than the LDS arrays hold (sources are table entries)."""
    w = synth.workload(config, dims=dims, segments=segments, n_boxes=n)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    X, Y, Z = dims
    boxes[:4] = [[0, 0, 0, X, Y, Z], [X - 1, Y - 1, Z - 1, 1, 1, 1], [1, 2, 3, X - 1, Y - 2, 1],
                 [0, 3, 0, X, 1, Z]]
    g = _graph(("runs", config, dims, segments), vol)
    _lut(g)
    assert g.info()["runs_mask"] & 3, "level 0 keeps no row runs"
    S = g.info()["nseg"]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    nnz = int((ref > 0).sum())
    try:
        for rm in (1, 0, 0xFFFFFFFF):
            g.set_launch_config(run_min_row=rm)
            for v in ("batched", "plain", "lut"):
                _compare(g.query(db, variant=v).cpu().numpy(), ref, l0, "run_min %d %s" % (rm, v))
            index, seg, val, total = g.query_sparse(db, capacity=nnz)
            assert int(total.item()) == nnz
            dense = _sparse_to_dense(index.cpu().numpy(), seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S)
            _compare(dense, ref, l0, "run_min %d sparse" % rm)
        g.set_launch_config(run_min_row=1, table_big=64, table_small=64, table_retry=64)
        _compare(g.query(db).cpu().numpy(), ref, l0, "runs, tiny tables")
    finally:
        g.set_launch_config(run_min_row=0, table_big=0, table_small=0, table_retry=0)


@pytest.mark.parametrize("nseg,dims", [(3, (96, 80, 64)), (7, (130, 70, 40))])
def test_query_on_noise_fills_the_deferred_run_rings(nseg, dims):
    """Uniform noise over a few segments: nearly every cube above level 0 is an internal node,
    so each wave step appends up to 64 deferred runs (the ring's fullest case) and rank-1 nodes
    carry every whole-voxel weight of their level; rank 2 and higher appear too. The batched,
    plain and lookup-table queries all give the oracle's histograms (noise keeps no row runs:
    its runs are too short, so every slab streams)."""
    vol = np.random.default_rng(nseg).integers(0, nseg, size=dims[::-1]).astype(np.uint32)
    g = _graph(("noise", nseg, dims), vol)
    _lut(g)
    X, Y, Z = dims
    rng = np.random.default_rng(1)
    lo = rng.integers(0, [X, Y, Z], size=(400, 3))
    ext = np.maximum(1, (rng.random((400, 3)) * ([X, Y, Z] - lo)).astype(np.int64))
    boxes = np.concatenate([lo, ext], axis=1).astype(np.uint32)
    boxes[:3] = [[0, 0, 0, X, Y, Z], [1, 3, 2, X - 1, Y - 3, Z - 2], [2, 0, 0, X - 2, Y, Z]]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    assert g.info()["runs_mask"] == 0
    for v in ("batched", "plain", "lut"):
        _compare(g.query(db, variant=v).cpu().numpy(), ref, l0, "noise %s" % v)


def test_query_edge_cases():
    vol = synth.make_volume(synth.workload(2, dims=(33, 35, 31), segments=25))
    nx, ny, nz = 33, 35, 31
    g = _graph("edge", vol)
    M = 0xFFFFFFFF
    boxes = np.array([
        [0, 0, 0, nx, ny, nz],          # full volume
        [5, 6, 7, 1, 1, 1],             # one voxel
        [nx, 0, 0, 4, 4, 4],            # origin at the x extent: empty
        [M, M, M, 4, 4, 4],             # far outside: empty
        [3, 3, 3, 0, 5, 5],             # zero extent: empty
        [10, 11, 12, M, M, M],          # huge extents clip
        [0, 0, 0, 1, ny, nz],           # one-voxel-thick slab
        [31, 0, 0, 2, 32, 16],          # aligned power-of-two block, clipped in x
        [1, 1, 1, 31, 33, 29],
    ], dtype=np.uint32)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    for v in ("batched", "plain", "naive"):
        out = g.query(_dev(boxes), variant=v).cpu().numpy()
        _compare(out, ref, None, v)
        assert (out[2:5] == 0).all()
        assert out[1].tolist() == [1.0 if s == vol_c[7, 6, 5] else 0.0 for s in range(len(ids))]
    # repeated calls with different sizes reuse the workspace
    for n in (1, 3, 9, 2):
        out = g.query(_dev(boxes[:n])).cpu().numpy()
        _compare(out, ref[:n], None, "n=%d" % n)
    empty = g.query(_dev(np.zeros((0, 6), dtype=np.uint32)))
    assert tuple(empty.shape) == (0, len(ids))


def test_query_bad_arguments():
    vol = synth.make_volume(synth.workload(2, dims=(16, 16, 16), segments=5))
    g = _graph("bad", vol)
    boxes = _dev(np.zeros((4, 6), dtype=np.uint32))
    out = torch.empty((4, g.info()["nseg"]), dtype=torch.float32, device="cuda")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(MGError) as e:
        g.query(boxes, out=out, workspace=small)
    assert e.value.code == -1


def test_query_full_config2_sampled():
    """512^3, 100,000 boxes, batched as bench.py runs it; O1 on a sample that includes the largest boxes."""
    w = synth.workload(2)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    g = _graph("cfg2", vol)
    db = _dev(boxes)
    out = g.query(db, variant="batched")
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    vols = boxes[:, 3:].astype(np.float64).prod(axis=1)
    sample = np.unique(np.concatenate([np.argsort(vols)[-40:], np.random.default_rng(7).choice(len(boxes), 160, replace=False)]))
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes[sample])
    _compare(got[sample], ref, None, "cfg2 sample")
    assert (got >= 0).all()
    assert np.abs(got.astype(np.float64).sum(axis=1) - 1.0).max() < 1e-5
    # the plain per-box kernel and the naive scan agree on the same sample
    for v in ("plain", "naive"):
        o = g.query(_dev(boxes[sample]), variant=v).cpu().numpy()
        _compare(o, ref, None, "cfg2 sample " + v)


# ------------------------------------------------------------------ TF propagation (a8)

@pytest.mark.parametrize("dims,segments", [((40, 36, 12), 30), ((72, 64, 40), 400)])
def test_tf_matches_oracle_every_mip_voxel(dims, segments):
    """Every node's colour at every mip voxel against the oracle's mean TF colour. With the
    deferred schedule the first volume's steps after the first are all small (one workgroup runs
    them); the second has steps of more than 4096 node x TF pairs (one launch each) before its
    small last steps. Rank by rank, both volumes have large first ranks and small last ones.
    Rank by rank, the first launch also computes rank 2, rebuilding the colours of rank-1
    predecessors from their sources; the deferred order reads them as stored, so equal colours
    across the two orders pin that rebuild bit for bit."""
    vol = synth.make_volume(synth.workload(3, dims=dims, segments=segments))
    g = _graph("tf%d" % segments, vol)
    inf = g.info()
    S = inf["nseg"]
    dag = g.export_dag()
    rp = np.asarray(dag["rank_ptr"])
    r2 = np.arange(rp[2], rp[3])
    for side in ("child_a", "child_b"):   # rank-2 nodes with rank-1 predecessors on either side
        p = np.asarray(dag[side])[r2]
        assert ((p >= rp[1]) & (p < rp[2])).any(), side
    steps = np.diff(dag["step_ptr"])[1:]
    if segments == 400:
        assert steps.max() * 5 > 4096 and steps[-1] * 5 <= 4096, steps
    tfs = synth.make_tfs(synth.workload(3), S, 5)
    ids, vol_c = scan.compact(vol)
    atol = 4 * max(inf["depth"], 1) * 2.0 ** -24
    want = [[None] * inf["n_levels"] for _ in range(5)]
    for l in range(inf["n_levels"]):   # the oracle's level colours, mixtures computed once per level
        h = mipmap.mixtures_level(vol_c, S, l)
        for t in range(5):
            want[t][l] = h @ otf.rgba_to_float(tfs[t])
    first = None
    # transfer functions per thread (5 planes: the last thread row is ragged) and the order of the
    # launches (rank by rank, or the deferred step schedule): launch knobs, never a change of colours
    for sched, planes in ((0, 0), (0, 1), (0, 2), (0, 4), (0, 8), (1, 0), (1, 1), (1, 8)):
        g.set_launch_config(tf_planes=planes, tf_schedule=sched)
        col = g.propagate_tf(torch.from_numpy(tfs).cuda()).cpu().numpy()
        for t in range(5):
            for l in range(inf["n_levels"]):
                got = col[t][g.export_map(l)].astype(np.float64)
                assert np.abs(got - want[t][l]).max() <= atol, (sched, planes, t, l, np.abs(got - want[t][l]).max())
        if first is None:
            first = col
        assert np.array_equal(col, first), (sched, planes)   # same arithmetic per node and plane
    g.set_launch_config(tf_planes=0, tf_schedule=0)
    with pytest.raises(MGError):
        g.set_launch_config(tf_planes=3)
    with pytest.raises(MGError):
        g.set_launch_config(tf_schedule=2)


def test_tf_frame_replays_and_capture():
    """Repeated frames on the same buffers, with eager work and synchronisations in between, equal
    the first frame bit for bit, as does a frame into new buffers; a frame captured into the
    caller's HIP graph replays to the same colours (the capture holds no memset); all agree with
    the oracle."""
    vol = synth.make_volume(synth.workload(3, dims=(72, 64, 40), segments=400))
    g = _graph("tf400", vol)
    inf = g.info()
    S, N = inf["nseg"], inf["n_nodes"]
    tfs = torch.from_numpy(synth.make_tfs(synth.workload(3), S, 3)).cuda()
    out = torch.empty((3, N, 4), dtype=torch.float32, device="cuda")
    g.propagate_tf(tfs, out=out)
    torch.cuda.synchronize()
    first = out.clone()
    ids, vol_c = scan.compact(vol)
    want = otf.level_colours(vol_c, S, tfs[1].cpu().numpy(), 1)
    got = first[1].cpu().numpy()[g.export_map(1)].astype(np.float64)
    assert np.abs(got - want).max() <= 4 * max(inf["depth"], 1) * 2.0 ** -24
    scratch = torch.ones(1 << 20, device="cuda")
    for k in range(4):
        out.zero_()
        scratch.mul_(1.5)
        g.propagate_tf(tfs, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, first), k
    other = torch.zeros_like(out)
    g.propagate_tf(tfs, out=other)
    torch.cuda.synchronize()
    assert torch.equal(other, first)
    cap = torch.zeros_like(out)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        g.propagate_tf(tfs, out=cap)   # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.propagate_tf(tfs, out=cap)
    for k in range(3):
        cap.zero_()
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(cap, first), k


def test_tf_constant_is_exact_and_one_hot_gives_mixture():
    vol = synth.make_volume(synth.workload(2, dims=(30, 30, 30), segments=40))
    g = _graph("tf2", vol)
    inf = g.info()
    S, N = inf["nseg"], inf["n_nodes"]
    const = np.tile(np.array([[17, 99, 250, 3]], dtype=np.uint8), (S, 1))[None]
    col = g.propagate_tf(torch.from_numpy(const).cuda()).cpu().numpy()
    assert (col[0] == (const[0, 0].astype(np.float32) * np.float32(1 / 255))).all()
    onehot = np.zeros((1, S, 4), dtype=np.uint8)
    onehot[0, 7, 0] = 255
    col = g.propagate_tf(torch.from_numpy(onehot).cuda()).cpu().numpy()[0, :, 0]
    ids, vol_c = scan.compact(vol)
    for l in range(inf["n_levels"]):
        h = mipmap.mixtures_level(vol_c, S, l)[..., 7]
        assert np.abs(col[g.export_map(l)] - h).max() <= 4 * inf["depth"] * 2.0 ** -24


def test_adjoint_box_colour():
    """Mean box colour two ways: sum_s p_s TF_s from the query, and sum over cubes of 8^l v_node / |box|
    from the propagated palette (the push is the transpose of the propagation)."""
    w = synth.workload(5, dims=(70, 64, 50), segments=60, n_boxes=300)
    vol = synth.make_volume(w)
    g = _graph("adj", vol)
    S = g.info()["nseg"]
    tf = synth.make_tfs(w, S, 1)
    boxes = synth.make_boxes(w)
    db = _dev(boxes)
    p = g.query(db).cpu().numpy().astype(np.float64)
    pal = g.propagate_tf(torch.from_numpy(tf).cuda()).cpu().numpy()[0].astype(np.float64)
    _, cubes = g.footprint(db, cubes_cap=4_000_000)
    cubes = cubes.cpu().numpy().astype(np.int64)
    acc = np.zeros((len(boxes), 4))
    np.add.at(acc, cubes[:, 0], (8.0 ** cubes[:, 1])[:, None] * pal[cubes[:, 5]])
    vols = np.prod(np.minimum(boxes[:, :3].astype(np.int64) + boxes[:, 3:], [70, 64, 50]) - boxes[:, :3], axis=1)
    lhs = p @ (tf[0].astype(np.float64) / 255.0)
    rhs = acc / vols[:, None]
    assert np.abs(lhs - rhs).max() < 1e-5


@pytest.mark.parametrize("dims", [(70, 64, 50), (200, 180, 60)])
def test_box_colour_kernel_is_the_cube_sum(dims):
    """mg_box_colour against the mean colour summed over the footprint cubes on the host (slabs
    of up to 36,000 cubes: several strides of the kernel's 1,024 threads x 8 cubes); rows without
    a palette get zeros."""
    w = synth.workload(5, dims=dims, segments=60, n_boxes=400)
    vol = synth.make_volume(w)
    g = _graph(("colour", dims), vol)
    S = g.info()["nseg"]
    tf = synth.make_tfs(w, S, 2)
    boxes = synth.make_boxes(w)
    X, Y, Z = dims
    boxes[:3] = [[0, 0, 0, X, Y, Z], [1, 1, 1, X - 2, Y - 2, Z - 2], [0, 0, 3, X, Y, 1]]
    db = _dev(boxes)
    pal = g.propagate_tf(torch.from_numpy(tf).cuda())
    pal_np = pal.cpu().numpy().astype(np.float64)
    which = (np.arange(len(boxes)) % 3).astype(np.int32)
    which[which == 2] = -1
    col = g.box_colour(pal, db, torch.from_numpy(which).cuda()).cpu().numpy().astype(np.float64)
    _, cubes = g.footprint(db, cubes_cap=40_000_000)
    cubes = cubes.cpu().numpy().astype(np.int64)
    acc = np.zeros((len(boxes), 4))
    t = which[cubes[:, 0]]
    keep = t >= 0
    np.add.at(acc, cubes[keep, 0], (8.0 ** cubes[keep, 1])[:, None] * pal_np[t[keep], cubes[keep, 5]])
    vols = np.prod(np.minimum(boxes[:, :3].astype(np.int64) + boxes[:, 3:], dims) - boxes[:, :3], axis=1)
    want = acc / vols[:, None]
    assert np.abs(col - want).max() < 1e-6
    assert (col[which < 0] == 0).all()


# ------------------------------------------------------------------ launch configurations (autotuner)

@pytest.mark.parametrize("ub,us,un,bs,bb", [(4, 16, 4, 256, 512), (16, 4, 16, 128, 256), (8, 8, 8, 128, 512),
                                            (8, 16, 8, 0, 256), (16, 8, 16, 256, 0)])
def test_query_every_unroll_variant(ub, us, un, bs, bb):
    w = synth.workload(2, dims=(150, 140, 130), segments=200, n_boxes=1500)
    vol = synth.make_volume(w)
    g = _graph(("unroll", ub, us, un), vol)
    g.set_launch_config(unroll_big=ub, unroll_small=us, unroll_naive=un, block_small=bs, block_big=bb)
    boxes = synth.make_boxes(w)
    boxes[:5] = [0, 0, 0, 150, 140, 130]          # big-tier boxes
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    for v in ("batched", "naive"):
        _compare(g.query(db, variant=v).cpu().numpy(), ref, None,
                 "%s u=%d/%d/%d b=%d/%d" % (v, ub, us, un, bs, bb))


def test_autotune_and_launch_validation():
    w = synth.workload(2, dims=(64, 64, 64), segments=40, n_boxes=500)
    vol = synth.make_volume(w)
    g = _graph("tune", vol)
    boxes = synth.make_boxes(w)
    db = _dev(boxes)
    cfg = g.autotune(db, reps=1)
    assert cfg["unroll_big"] in (4, 8, 16) and cfg["unroll_small"] in (4, 8, 16)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    _compare(g.query(db).cpu().numpy(), ref, None, "after autotune")
    with pytest.raises(MGError) as e:
        g.set_launch_config(unroll_big=5)
    assert e.value.code == -1
    with pytest.raises(MGError):
        g.set_launch_config(tf_block=100)
    with pytest.raises(MGError):
        g.set_launch_config(block_small=192)
    with pytest.raises(MGError):
        g.set_launch_config(block_big=128)
    with pytest.raises(MGError):
        g.set_launch_config(chunk_small=65)
    assert g.launch_config() == cfg
    # boxes per dequeue of the small tier: a scheduling knob, never a change of results
    for c in (1, 3, 64, 0):
        g.set_launch_config(chunk_small=c)
        _compare(g.query(db).cpu().numpy(), ref, None, "chunk_small %d" % c)
    g.set_launch_config(**cfg)


def test_overflow_retry_and_global_fallback_paths():
    """Tiny LDS tables force boxes through the retry launch and the global-memory fallback;
    results must not change (the table sizes are a launch knob set from the host)."""
    w = synth.workload(2, dims=(160, 150, 140), segments=300, n_boxes=800)
    vol = synth.make_volume(w)
    g = _graph("ovf", vol)
    boxes = synth.make_boxes(w)
    boxes[:10] = [0, 0, 0, 160, 150, 140]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    for tb, ts, tr in ((64, 64, 8192), (64, 64, 64), (4096, 1024, 0)):
        g.set_launch_config(table_big=tb, table_small=ts, table_retry=tr)
        out, stats = g.query_stats(db)
        st = stats.cpu().numpy().view(np.uint32)
        _compare(out.cpu().numpy(), ref, None, "tables %d/%d/%d" % (tb, ts, tr))
        via_retry = int(((st[:, 1] >> 30) & 1).sum())
        via_global = int((st[:, 1] >> 31).sum())
        if tr == 8192:
            assert via_retry > 0 and via_global == 0
        if tr == 64:
            assert via_global > 0
    for v in ("plain",):
        g.set_launch_config(table_big=0, table_small=0, table_retry=64)
        _compare(g.query(db, variant=v).cpu().numpy(), ref, None, "plain with tiny retry table")
    g.set_launch_config(table_big=0, table_small=0, table_retry=0)


def test_mid_size_global_tables():
    """A graph larger than one mid-size global table (65,536 slots) with tiny LDS tables: boxes
    overflow every LDS table and are answered by the many-worker mid-size global tables (with
    per-source arrays), the largest ones by the whole-graph tables; dense rows and sparse entries
    match the oracle."""
    w = synth.workload(4, dims=(150, 170, 160), segments=5000, n_boxes=700)
    vol = synth.make_volume(w)
    g = Graph.build(vol).upload(0)
    inf = g.info()
    assert inf["n_nodes"] * 4 // 3 + 2 > 65536, inf["n_nodes"]
    S = inf["nseg"]
    boxes = synth.make_boxes(w)
    boxes[:4] = [[0, 0, 0, 150, 170, 160], [1, 2, 3, 140, 160, 150], [149, 169, 159, 1, 1, 1], [9, 9, 9, 0, 3, 3]]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, S, boxes)
    db = _dev(boxes)
    g.set_launch_config(table_big=64, table_small=64, table_retry=64)
    out, stats = g.query_stats(db)
    st = stats.cpu().numpy().view(np.uint32)
    assert int((st[:, 1] >> 31).sum()) > 100
    _compare(out.cpu().numpy(), ref, None, "mid-size global tables, dense rows")
    nnz = int((ref > 0).sum())
    want = (ref > 0).sum(axis=1)
    for tables in ((0, 0, 0), (64, 64, 64)):
        g.set_launch_config(table_big=tables[0], table_small=tables[1], table_retry=tables[2])
        index, seg, val, total = g.query_sparse(db, capacity=nnz)
        idx = index.cpu().numpy().astype(np.int64)
        bad = np.nonzero(idx[:, 1] != want)[0]
        assert len(bad) == 0, "tables %s: %d boxes with wrong entry counts, e.g. %s" % (
            tables, len(bad), [(int(q), int(idx[q, 1]), int(want[q]), int(st[q, 1] >> 30), int(st[q, 0]))
                               for q in bad[:6]])
        assert int(total.item()) == nnz
        dense = _sparse_to_dense(idx, seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S)
        _compare(dense, ref, None, "sparse entries, tables %s" % (tables,))
    g.set_launch_config(table_big=0, table_small=0, table_retry=0)
    _compare(g.query(db).cpu().numpy(), ref, None, "default tables")
    g.close()


# ------------------------------------------------------------------ many segments: sources in the table

def _sparse_to_dense(index, seg, val, n, S):
    out = np.zeros((n, S), dtype=np.float64)
    index = index.astype(np.int64)
    for q in range(n):
        b, k = index[q]
        assert b >= 0 and k >= 0
        s_ = seg[b:b + k]
        assert len(np.unique(s_)) == len(s_)           # each segment once per box
        out[q, s_] = val[b:b + k]
    return out


def test_query_many_segments_dense_and_sparse():
    """More sources than the LDS arrays hold (cylinder recipe, > 2048 segments): sources become table
    entries; dense rows and the sparse entry list both match the oracle."""
    w = synth.workload(4, dims=(160, 200, 150), segments=4000, n_boxes=1500)
    vol = synth.make_volume(w)
    g = _graph("many", vol)
    S = g.info()["nseg"]
    assert S > 2048
    boxes = synth.make_boxes(w)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    for v in ("batched", "plain", "naive"):
        _compare(g.query(db, variant=v).cpu().numpy(), ref, l0, "many segments " + v)
    nnz = int((ref > 0).sum())
    index, seg, val, total = g.query_sparse(db, capacity=nnz + 10)
    assert int(total.item()) == nnz
    dense = _sparse_to_dense(index.cpu().numpy(), seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S)
    _compare(dense, ref, l0, "sparse output")


def test_query_more_sources_than_16_bit_ids():
    """70,001 sources (more than a 16-bit ID holds): no 16-bit level-0 copy, sources are table
    entries, depth 17; dense rows and sparse entries match the oracle, the naive scan (per-source
    LDS counters) refuses with MG_ELIMIT."""
    Z, Y, X = 48, 64, 64
    blocks = np.arange(Z * Y * (X // 2)).reshape(Z, Y, X // 2)
    vol = np.repeat((blocks * 7919) % 70001, 2, axis=2).astype(np.uint32)
    g = Graph.build(vol).upload(0)
    S = g.info()["nseg"]
    assert S == 70001
    rng = np.random.default_rng(11)
    boxes = np.concatenate([rng.integers(0, 40, size=(300, 3)), rng.integers(1, 30, size=(300, 3))],
                           axis=1).astype(np.uint32)
    boxes[0] = [0, 0, 0, X, Y, Z]
    boxes[1] = [5, 6, 7, 1, 1, 1]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, S, boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    for v in ("batched", "plain"):
        _compare(g.query(db, variant=v).cpu().numpy(), ref, l0, "70001 sources " + v)
    nnz = int((ref > 0).sum())
    index, seg, val, total = g.query_sparse(db, capacity=nnz)
    assert int(total.item()) == nnz
    dense = _sparse_to_dense(index.cpu().numpy(), seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S)
    _compare(dense, ref, l0, "70001 sources sparse")
    with pytest.raises(MGError) as e:
        g.query(db, variant="naive")
    assert e.value.code == -8


def test_query_sparse_output_small_segment_count_and_truncation():
    w = synth.workload(2, dims=(90, 80, 70), segments=120, n_boxes=700)
    vol = synth.make_volume(w)
    g = _graph("sparse_small", vol)
    S = g.info()["nseg"]
    boxes = synth.make_boxes(w)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    nnz = int((ref > 0).sum())
    index, seg, val, total = g.query_sparse(db, capacity=nnz)
    assert int(total.item()) == nnz
    _compare(_sparse_to_dense(index.cpu().numpy(), seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S), ref, None,
             "sparse")
    # too little room: the total still reports what was needed, and written entries are valid
    cap = nnz // 3
    index, seg, val, total = g.query_sparse(db, capacity=cap)
    assert int(total.item()) == nnz
    index, seg, val = index.cpu().numpy().astype(np.int64), seg.cpu().numpy(), val.cpu().numpy()
    for q in range(len(boxes)):
        b, k = index[q]
        for j in range(b, min(b + k, cap)):
            r = ref[q, seg[j]]
            assert r > 0 and abs(val[j] - r) <= REL_TOL * r


def test_nnz_bound_sizes_the_sparse_output():
    """mg_query_nnz_bound: for every box at least its non-zero segments (oracle counts), at most the
    source count and the box volume, 0 for empty boxes; a sparse query sized by the sum of the bounds
    does not truncate and matches the oracle."""
    w = synth.workload(4, dims=(150, 160, 140), segments=1500, n_boxes=900)
    vol = synth.make_volume(w)
    g = Graph.build(vol).upload(0)
    S = g.info()["nseg"]
    boxes = synth.make_boxes(w)
    boxes[:5] = [[0, 0, 0, 150, 160, 140], [149, 159, 139, 1, 1, 1], [7, 8, 9, 0, 5, 5],
                 [200, 0, 0, 5, 5, 5], [3, 3, 3, 1, 90, 1]]
    ids, vol_c = scan.compact(vol)
    cnt, ref = scan.box_counts(vol_c, S, boxes)
    db = _dev(boxes)
    bound = g.nnz_bound(db).cpu().numpy().astype(np.int64)
    nnz = (ref > 0).sum(axis=1)
    b = boxes.astype(np.int64)
    dims = np.array(w.dims)
    vols = np.prod(np.maximum(np.minimum(b[:, :3] + b[:, 3:], dims) - np.minimum(b[:, :3], dims), 0), axis=1)
    assert (bound >= nnz).all(), np.nonzero(bound < nnz)[0][:5]
    assert (bound <= np.minimum(S, vols)).all()
    assert bound[2] == 0 and bound[3] == 0 and bound[1] == 1
    cap = int(bound.sum())
    index, seg, val, total = g.query_sparse(db, capacity=cap)
    assert int(total.item()) == int(nnz.sum()) <= cap
    dense = _sparse_to_dense(index.cpu().numpy(), seg.cpu().numpy(), val.cpu().numpy(), len(boxes), S)
    _compare(dense, ref, None, "sparse output sized by the bound")
    g.close()


def test_bind_device_into_a_caller_buffer():
    """mg_bind_device: the graph's arrays in a torch-owned buffer answer exactly like mg_upload's copy
    (queries against the oracle, TF propagation equal), and small or misaligned buffers are refused."""
    w = synth.workload(2, dims=(120, 110, 100), segments=200, n_boxes=600)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    g_up = Graph.build(vol).upload(0)
    g = Graph.build(vol)
    nbytes = g.device_bytes()
    with pytest.raises(MGError) as e:
        g.bind(torch.empty(nbytes - 256, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -1
    big = torch.empty(nbytes + 512, dtype=torch.uint8, device="cuda")
    with pytest.raises(MGError) as e:
        g.bind(big[4:4 + nbytes])
    assert e.value.code == -1
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    g.bind(buf)
    assert g.info()["device"] == 0 and g.info()["device_bytes"] == nbytes
    out = g.query(db).cpu().numpy()
    _compare(out, ref, None, "bound buffer")
    assert np.array_equal(g.query(db, variant="naive").cpu().numpy(), g_up.query(db, variant="naive").cpu().numpy())
    S = len(ids)
    tf = torch.from_numpy(synth.make_tfs(w, S, 2)).cuda()
    assert torch.equal(g.propagate_tf(tf), g_up.propagate_tf(tf))
    g.close()
    g_up.close()
    del buf


# ------------------------------------------------------------------ serving loop (continuous batching)

def _served(w, n, qps, arrivals=None, **kw):
    from paper_2009_02702_amd.serve import Server
    vol = synth.make_volume(w)
    g = _graph(("serve", w.dims), vol)
    S = g.info()["nseg"]
    boxes = synth.make_boxes(w, n)
    if arrivals is None:
        arrivals = synth.poisson_arrivals(w, n, qps)
    tf_index = np.full(n, -1, dtype=np.int64)
    tf_rows = np.arange(0, n, 10)
    tf_index[tf_rows] = np.arange(len(tf_rows))
    tfs = synth.make_tfs(w, S, len(tf_rows))
    srv = Server(g, **kw)
    res = np.zeros((n, S), dtype=np.float32)
    col = np.full((n, 4), np.nan, dtype=np.float64)
    stats = srv.serve(boxes, arrivals, tf_index, tfs, results=res, colours=col)
    _served.last = {"tf_index": tf_index, "tfs": tfs, "colours": col}
    return g, boxes, res, stats


def _check_served_colours(boxes, ref, tag):
    """Each TF request's served box colour (from its propagated palette, over the box's footprint
    cubes) equals the mean TF colour over the box's voxels: sum_s p_s TF_s / 255 from the oracle's
    fractions (the adjoint of the push). Other requests get no colour."""
    last = _served.last
    ti, tfs, col = last["tf_index"], last["tfs"], last["colours"]
    has = ti >= 0
    assert np.isnan(col[~has]).all(), tag
    want = np.einsum("qs,qsc->qc", ref[has], tfs[ti[has]].astype(np.float64) / 255.0)
    empty = ref[has].sum(axis=1) == 0
    want[empty] = 0.0
    assert np.isfinite(col[has]).all(), tag
    assert np.abs(col[has] - want).max() <= 1e-5, "%s: colour err %g" % (tag, np.abs(col[has] - want).max())


def test_serving_results_equal_alone_and_in_the_mix():
    """Every served result (admitted in batches that overlap on several streams, replayed from
    captured graphs) matches the same box queried alone, and the oracle; every TF request's box
    colour matches the oracle's mean colour and the same colouring run alone."""
    w = synth.workload(5, dims=(140, 130, 100), segments=80)
    g, boxes, res, stats = _served(w, 3000, 20000.0, slots=3, max_batch=256, max_tf=8)
    assert np.isfinite(stats.latency_s).all() and (stats.latency_s >= 0).all()
    assert stats.batches > 1
    ids, vol_c = scan.compact(synth.make_volume(w))
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    _compare(res, ref, None, "served")
    alone = np.stack([g.query(_dev(boxes[i:i + 1])).cpu().numpy()[0] for i in range(0, 3000, 97)])
    _compare(res[::97], alone.astype(np.float64), None, "served vs alone")
    _check_served_colours(boxes, ref, "served colours")
    # the same colouring alone: propagate request 0's TF and colour its box on the default stream
    last = _served.last
    i0 = int(np.nonzero(last["tf_index"] >= 0)[0][0])
    pal = g.propagate_tf(torch.from_numpy(last["tfs"][last["tf_index"][i0]][None].copy()).cuda())
    one = g.box_colour(pal, _dev(boxes[i0:i0 + 1]), torch.zeros(1, dtype=torch.int32, device="cuda"))
    assert np.abs(one.cpu().numpy()[0] - last["colours"][i0]).max() <= 1e-6
    s = stats.summary()
    assert s["batch_ms"]["device_max"] > 0
    print(s)


def test_serving_full_batches_above_every_default_class():
    """max_batch outside the default size classes (512) with every request arriving at once, so
    batches fill to max_batch: every row is answered (a regression test for batches larger than
    the largest captured graph)."""
    w = synth.workload(5, dims=(120, 100, 90), segments=60)
    n = 2000
    g, boxes, res, stats = _served(w, n, 1.0, arrivals=np.zeros(n), slots=2, max_batch=512, max_tf=64,
                                   split_cubes=1 << 30)
    assert max(stats.batch_sizes) == 512
    ids, vol_c = scan.compact(synth.make_volume(w))
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    _compare(res, ref, None, "full batches")
    _check_served_colours(boxes, ref, "full batches colours")


def test_serving_rejects_tf_requests_without_tf_slots():
    from paper_2009_02702_amd.serve import Server
    w = synth.workload(5, dims=(60, 50, 40), segments=20)
    g = _graph(("serve", w.dims), synth.make_volume(w))
    srv = Server(g, slots=1, max_batch=64, max_tf=0, use_graphs=False)
    boxes = synth.make_boxes(w, 10)
    ti = np.full(10, -1)
    ti[0] = 0
    with pytest.raises(ValueError):
        srv.serve(boxes, np.zeros(10), ti, synth.make_tfs(w, g.info()["nseg"], 1))
    st = srv.serve(boxes, np.zeros(10))   # boxes alone still work
    assert st.batches >= 1


def test_serving_splits_big_boxes_into_sub_boxes():
    """Boxes above the split threshold are answered as aligned sub-boxes in the same batch and
    recombined by volume: the result still matches the oracle (tiny thresholds force splits)."""
    from paper_2009_02702_amd.serve import cube_counts, split_box
    w = synth.workload(2, dims=(120, 110, 90), segments=70)
    g, boxes, res, stats = _served(w, 600, 5000.0, slots=2, max_batch=512, max_tf=8, split_cubes=2000,
                                   piece_cubes=700)
    cubes = cube_counts(boxes, w.dims)
    assert (cubes >= 2000).sum() > 50          # many requests were split
    big = boxes[np.argmax(cubes)].astype(np.int64)
    sub = split_box(big, w.dims, 8)
    clipped = np.prod(np.minimum(big[:3] + big[3:], w.dims) - big[:3])
    assert len(sub) > 1 and np.prod(sub[:, 3:].astype(np.int64), axis=1).sum() == clipped
    ids, vol_c = scan.compact(synth.make_volume(w))
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    _compare(res, ref, None, "served with splits")
    _check_served_colours(boxes, ref, "served with splits colours")


def test_serving_small_budget_queues_instead_of_failing():
    from paper_2009_02702_amd.serve import Server
    w = synth.workload(5, dims=(100, 90, 80), segments=40)
    g = _graph(("serve", w.dims), synth.make_volume(w))
    one = Server(g, slots=1, max_batch=1, max_tf=1, use_graphs=False).device_bytes
    g2, boxes, res, stats = _served(w, 400, 50000.0, slots=4, max_batch=512, max_tf=4,
                                    budget_bytes=one * 3, use_graphs=False)
    assert max(stats.batch_sizes) <= 512
    ids, vol_c = scan.compact(synth.make_volume(w))
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    _compare(res, ref, None, "small budget")
    with pytest.raises(ValueError):
        Server(g, budget_bytes=16)


# ------------------------------------------------------------------ mixture lookup table query and palette fetch

def test_lut_query_config1_full():
    _, errs = _check_workload(synth.workload(1), variants=("lut",))
    print(errs)


@pytest.mark.parametrize("config,dims,segments,n", [
    (2, (96, 80, 72), 353, 3000),
    (3, (256, 256, 40), 1182, 2000),
    (4, (123, 96, 100), 1500, 3000),
    (5, (118, 113, 79), 353, 3000),
])
def test_lut_query_reduced_recipes(config, dims, segments, n):
    _, errs = _check_workload(synth.workload(config, dims=dims, segments=segments, n_boxes=n), variants=("lut",))
    print(errs)


def test_lut_query_many_segments_and_tiny_tables():
    """Sources as table entries (> 2048 segments), and tables small enough to force the retry and
    global-memory launches: the lookup-table expansion gives the oracle's histograms on every path."""
    w = synth.workload(4, dims=(160, 200, 150), segments=4000, n_boxes=1500)
    vol = synth.make_volume(w)
    g = _lut(_graph("many", vol))
    boxes = synth.make_boxes(w)
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    _compare(g.query(db, variant="lut").cpu().numpy(), ref, _level0_only(g, db), "many segments lut")
    w = synth.workload(2, dims=(160, 150, 140), segments=300, n_boxes=800)
    vol = synth.make_volume(w)
    g = _lut(_graph("ovf", vol))
    boxes = synth.make_boxes(w)
    boxes[:10] = [0, 0, 0, 160, 150, 140]
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    for tb, ts, tr in ((64, 64, 8192), (64, 64, 64)):
        g.set_launch_config(table_big=tb, table_small=ts, table_retry=tr)
        _compare(g.query(db, variant="lut").cpu().numpy(), ref, None, "lut tables %d/%d/%d" % (tb, ts, tr))
    g.set_launch_config(table_big=0, table_small=0, table_retry=0)


def test_lut_query_needs_the_table():
    g = Graph.build(synth.make_volume(synth.workload(2, dims=(20, 20, 20), segments=10))).upload(0)
    with pytest.raises(MGError) as e:
        g.query(_dev(np.array([[0, 0, 0, 5, 5, 5]], dtype=np.uint32)), variant="lut")
    assert e.value.code == -4


@pytest.mark.parametrize("factorizer,tau", [("reduction", 3), ("occurrence", 3), ("reduction", 0)])
def test_query_on_greedy_factorized_graphs(factorizer, tau):
    """Graphs from the paper's greedy factorizer (deeper, different shape) answer every box like O1,
    through the batched push, the plain kernel and the lookup table."""
    w = synth.workload(2, dims=(96, 90, 80), segments=120, n_boxes=600)
    vol = synth.make_volume(w)
    boxes = synth.make_boxes(w)
    boxes[0] = [0, 0, 0, 96, 90, 80]
    g = Graph.build(vol, factorizer=factorizer, tau=tau).upload(0)
    g.lut_build()
    ids, vol_c = scan.compact(vol)
    _, ref = scan.box_counts(vol_c, len(ids), boxes)
    db = _dev(boxes)
    l0 = _level0_only(g, db)
    for v in ("batched", "plain", "lut"):
        _compare(g.query(db, variant=v).cpu().numpy(), ref, l0, "greedy %s/%s" % (factorizer, v))


def test_palette_fetch_is_the_palette_at_the_voxel_node():
    """Paletted fetch (Sec. 'Rendering'): colour of a mip voxel = palette[node of the voxel], bit for bit;
    coordinates outside the level give zeros; the fetched colour is the mean TF over the voxel's support."""
    vol = synth.make_volume(synth.workload(3, dims=(40, 36, 12), segments=30))
    g = _graph("tf", vol)
    inf = g.info()
    S = inf["nseg"]
    tfs = synth.make_tfs(synth.workload(3), S, 2)
    pal = g.propagate_tf(torch.from_numpy(tfs).cuda())
    pal_h = pal.cpu().numpy()
    ids, vol_c = scan.compact(vol)
    rng = np.random.default_rng(5)
    atol = 4 * max(inf["depth"], 1) * 2.0 ** -24
    for l in (0, 1, 3, inf["n_levels"] - 1):
        m = g.export_map(l)                       # [Z, Y, X]
        Z, Y, X = m.shape
        xyz = np.stack([rng.integers(0, X + 2, 500), rng.integers(0, Y + 2, 500), rng.integers(0, Z + 2, 500)],
                       axis=1).astype(np.uint32)
        got = g.palette_fetch(pal, l, _dev(xyz)).cpu().numpy()
        inside = (xyz[:, 0] < X) & (xyz[:, 1] < Y) & (xyz[:, 2] < Z)
        assert (got[:, ~inside] == 0).all()
        xi = xyz[inside].astype(np.int64)
        node = m[xi[:, 2], xi[:, 1], xi[:, 0]]
        assert np.array_equal(got[:, inside], pal_h[:, node])
        for t in range(2):
            want = otf.level_colours(vol_c, S, tfs[t], l)[xi[:, 2], xi[:, 1], xi[:, 0]]
            assert np.abs(got[t, inside] - want).max() <= atol
    with pytest.raises(MGError):
        g.palette_fetch(pal, inf["n_levels"], _dev(np.zeros((1, 3), dtype=np.uint32)))
