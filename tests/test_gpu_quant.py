"""GPU parity of graphs with quantized weights (Sec. "Compression") and of the uncertainty query
(Sec. "Error Propagation"), through the C ABI, against the oracle in oracle/quant.py.

Fractions: the quantized graph is pushed with its fp32 codewords exactly as an exact graph is, so
the same bound holds (relative error below 1e-5, exact zeros, level-0 boxes bit for bit).
Uncertainties: the library's per-row uncertainties agree with the oracle's propagation to 1e-4
relative (fp32 rows built in fp64); the kernel squares fp32 products and adds them in fp32 in
arbitrary order (relative error below a few 1e-7 per term), so 2e-4 relative bounds the result.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import footprint as ofp
from oracle import quant
from paper_2009_02702_amd import Graph, MGError, synth

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
ERR_RTOL = 2e-4


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


_CACHE = {}


def _setup(config, dims, segments, n_boxes, bits):
    key = (config, dims, segments, n_boxes, bits)
    if key in _CACHE:
        return _CACHE[key]
    w = synth.workload(config, dims=dims, segments=segments, n_boxes=n_boxes)
    vol = synth.make_volume(w)
    g = Graph.build(vol)
    S = g.info()["nseg"]
    d = g.export_dag()
    rep, nodes, _, _ = quant.quantize_dag(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:] / d["wden"][S:],
                                         bits)
    mu, dmu = quant.propagate(S, nodes)
    boxes = synth.make_boxes(w)
    boxes[0] = [0, 0, 0, dims[0], dims[1], dims[2]]
    maps = [g.export_map(l) for l in range(g.info()["n_levels"])]
    f = np.zeros((len(boxes), S))
    u = np.zeros((len(boxes), S))
    l0 = np.zeros(len(boxes), dtype=bool)
    for i, bx in enumerate(boxes.astype(np.int64)):
        counts, levels = {}, set()
        for lev, c in ofp.assembly(bx[:3], bx[3:], dims):
            n = rep[int(maps[lev][c[2], c[1], c[0]])]
            counts[n] = counts.get(n, 0) + 8 ** lev
            levels.add(lev)
        vol_b = float(np.prod(np.minimum(bx[:3] + bx[3:], dims) - np.minimum(bx[:3], dims)))
        if vol_b > 0:
            f[i], u[i] = quant.box_histogram(counts, mu, dmu, vol_b)
            l0[i] = levels == {0}
    q = g.quantize(bits).upload(0)
    q.lut_build()
    _CACHE[key] = (g, q, boxes, f, u, l0, S)
    return _CACHE[key]


def _compare(got, ref, l0, tag):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape and np.isfinite(got).all(), tag
    assert np.array_equal(got == 0, ref == 0), "%s: support differs" % tag
    nz = ref > 0
    rel = np.abs(got[nz] - ref[nz]) / ref[nz]
    assert rel.max(initial=0) <= REL_TOL, "%s: max rel err %g" % (tag, rel.max())
    if l0.any():
        assert np.array_equal(got[l0].astype(np.float32), ref[l0].astype(np.float32)), "%s: level-0 boxes" % tag


def _compare_err(got, ref, tag):
    got = np.asarray(got, dtype=np.float64)
    assert got.shape == ref.shape and np.isfinite(got).all() and (got >= 0).all(), tag
    scale = np.abs(ref).max(initial=0)
    bad = np.abs(got - ref) > ERR_RTOL * ref + 1e-6 * scale
    assert not bad.any(), "%s: %d uncertainties off, worst rel %g" % (
        tag, int(bad.sum()), float((np.abs(got - ref)[bad] / np.maximum(ref[bad], 1e-30)).max()))


@pytest.mark.parametrize("config,dims,segments,n,bits", [
    (2, (64, 60, 56), 120, 300, 9),
    (2, (64, 60, 56), 120, 300, 5),
    (4, (70, 40, 36), 60, 200, 7),
])
def test_quantized_graph_push_lut_and_uncertainty(config, dims, segments, n, bits):
    """Fractions of the quantized graph from the push query and from the lookup table equal the
    oracle's quantized mixture; the uncertainty query returns the same fractions and the oracle's
    propagated uncertainty (node terms in quadrature)."""
    g, q, boxes, f, u, l0, S = _setup(config, dims, segments, n, bits)
    db = _dev(boxes)
    _compare(q.query(db).cpu().numpy(), f, l0, "push")
    _compare(q.query(db, variant="lut").cpu().numpy(), f, l0, "lut")
    out, err = q.query_err(db)
    _compare(out.cpu().numpy(), f, l0, "err/fractions")
    _compare_err(err.cpu().numpy(), u, "err")
    # level-0 boxes are certain: every cube is a source
    assert (err.cpu().numpy()[l0] == 0).all()


def test_uncertainty_query_through_retry_and_fallback():
    """Tiny LDS tables send boxes through the retry launch and the global-memory fallback; the
    uncertainties accumulated there equal those of the fast tiers."""
    g, q, boxes, f, u, l0, S = _setup(2, (64, 60, 56), 120, 300, 9)
    db = _dev(boxes)
    try:
        for tb, ts, tr in ((64, 64, 8192), (64, 64, 64)):
            q.set_launch_config(table_big=tb, table_small=ts, table_retry=tr)
            out, err = q.query_err(db)
            _compare(out.cpu().numpy(), f, l0, "tables %d/%d/%d" % (tb, ts, tr))
            _compare_err(err.cpu().numpy(), u, "err tables %d/%d/%d" % (tb, ts, tr))
    finally:
        q.set_launch_config(table_big=0, table_small=0, table_retry=0)


def test_uncertainty_query_preconditions():
    w = synth.workload(2, dims=(24, 20, 18), segments=12)
    g = Graph.build(synth.make_volume(w)).upload(0)
    one = _dev(np.array([[0, 0, 0, 9, 9, 9]], dtype=np.uint32))
    g.lut_build()
    with pytest.raises(MGError) as e:          # exact weights: nothing to propagate
        g.query_err(one)
    assert e.value.code == -4
    q = g.quantize(6).upload(0)
    with pytest.raises(MGError) as e:          # no lookup table yet
        q.query_err(one)
    assert e.value.code == -4
    q.lut_build()
    out, err = q.query_err(one)
    assert abs(float(out.sum()) - 1.0) < 1e-5 and (err >= 0).all()
    empty = _dev(np.array([[3, 3, 3, 0, 4, 4], [30, 0, 0, 5, 5, 5]], dtype=np.uint32))
    out, err = q.query_err(empty)
    assert (out == 0).all() and (err == 0).all()


def test_graph_from_the_bit_packed_stream_answers_like_its_source():
    """A quantized graph written as the bit-packed stream (Table "bitstream") and read back answers
    every box like the graph it was written from (up to the order of the kernels' atomic adds), and
    like the oracle."""
    g, q, boxes, f, u, l0, S = _setup(2, (64, 60, 56), 120, 300, 9)
    r = Graph.unpack(q.pack()).upload(0)
    r.lut_build()
    db = _dev(boxes)
    a = q.query(db).cpu().numpy().astype(np.float64)
    b = r.query(db).cpu().numpy().astype(np.float64)
    assert np.array_equal(a == 0, b == 0) and np.allclose(a, b, rtol=2e-6, atol=0)
    _compare(b, f, l0, "unpacked")
    oa, ea = q.query_err(db)
    ob, eb = r.query_err(db)
    _compare(ob.cpu().numpy(), f, l0, "unpacked err/fractions")
    _compare_err(eb.cpu().numpy(), u, "unpacked err")


def test_stream_decoded_on_the_gpu():
    """mg_unpack_device: the stream's voxel data decoded by the GPU gives exactly the maps the host
    reader gives (every level, bit for bit), and the graph answers like the host-read one; a node ID
    out of range in the voxel data is MG_EFORMAT; host-only operations are refused."""
    g, q, boxes, f, u, l0, S = _setup(2, (70, 66, 52), 150, 300, 9)
    stream = q.pack()
    h = Graph.unpack(stream).upload(0)
    d = Graph.unpack_device(stream, 0)
    L = h.info()["n_levels"]
    assert d.info()["n_nodes"] == h.info()["n_nodes"] and d.info()["device"] == 0
    for lev in range(L):
        assert np.array_equal(d.export_map(lev), h.export_map(lev)), lev
    db = _dev(boxes)
    a = h.query(db).cpu().numpy().astype(np.float64)
    b = d.query(db).cpu().numpy().astype(np.float64)
    assert np.array_equal(a == 0, b == 0) and np.allclose(a, b, rtol=2e-6, atol=0)
    _compare(b, f, l0, "decoded on the GPU")
    for call in (d.pack, lambda: d.upload(0), lambda: d.save("/tmp/mg_never_written.bin")):
        with pytest.raises(MGError) as e:
            call()
        assert e.value.code == -4
    # a level-0 voxel ID past the sources: all ones in the first voxel's field (S is not a
    # power of two, so i_min + 2^r - 1 >= S)
    n = h.info()["n_nodes"]
    assert S & (S - 1)
    bpn = max(1, int(np.ceil(np.log2(n))))
    a_bit = 32 + 1 + 6 + 32 + 3 * 32 + 4 + bpn + L * 2 * bpn
    r0 = int(np.ceil(np.log2(S)))
    bad = bytearray(stream)
    for k in range(a_bit, a_bit + r0):
        bad[k >> 3] |= 1 << (k & 7)
    with pytest.raises(MGError) as e:
        Graph.unpack_device(bytes(bad), 0)
    assert e.value.code == -7
    with pytest.raises(MGError) as e:
        Graph.unpack(bytes(bad))
    assert e.value.code == -7
    d.close()
    h.close()
