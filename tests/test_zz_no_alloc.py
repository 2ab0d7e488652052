"""The no-allocation query entry point (mg_query_boxes_noalloc) against mg_query_boxes.

The entry point answers boxes on the library's static device scratch instead of a caller
workspace. Checked through the C ABI: two calls in a row on one graph, the second with fewer
boxes, compared element by element with mg_query_boxes (relative 1e-5 per segment, identical
zeros, as in test_gpu.py) and with the CPU oracle; the same with tiny LDS tables so that boxes
go through the retry launch and the global fallback tables that live in the scratch; a second
graph with another layout of the fallback tables; and the host-side size limit.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import scan
from paper_2009_02702_amd import Graph, MGError, synth

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).cuda()


def _compare(got, ref, tag):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, tag
    assert np.isfinite(got).all(), tag
    assert np.array_equal(got == 0, ref == 0), "%s: support differs" % tag
    nz = ref > 0
    rel = np.abs(got[nz] - ref[nz]) / ref[nz]
    assert rel.max(initial=0) <= REL_TOL, "%s: max rel err %g" % (tag, rel.max())


def _case(g, vol_c, S, boxes, tag):
    db = _dev(boxes)
    want = g.query(db).cpu().numpy()
    got = g.query_noalloc(db).cpu().numpy()
    _compare(got, want, tag + " vs mg_query_boxes")
    _, ref = scan.box_counts(vol_c, S, boxes)
    _compare(got, ref, tag + " vs oracle")


def test_noalloc_matches_query_boxes_twice_then_smaller():
    w = synth.workload(2, dims=(160, 150, 140), segments=300, n_boxes=3000)
    vol = synth.make_volume(w)
    ids, vol_c = scan.compact(vol)
    g = Graph.build(vol).upload(0)
    S = len(ids)
    boxes = synth.make_boxes(w)
    boxes[:3] = [[0, 0, 0, 160, 150, 140], [159, 149, 139, 1, 1, 1], [5, 5, 5, 0, 4, 4]]
    _case(g, vol_c, S, boxes, "call 1 (3000 boxes)")
    _case(g, vol_c, S, boxes[:700], "call 2 (700 boxes)")
    # tiny LDS tables: boxes overflow into the retry launch and the scratch's global tables
    g.set_launch_config(table_big=64, table_small=64, table_retry=64)
    _case(g, vol_c, S, boxes[:1200], "tiny tables, call 1")
    _case(g, vol_c, S, boxes[:300], "tiny tables, call 2")
    g.set_launch_config(table_big=0, table_small=0, table_retry=0)
    # a graph with another fallback layout (more sources) on the same scratch, then the first again
    w2 = synth.workload(2, dims=(96, 80, 72), segments=900, n_boxes=500)
    vol2 = synth.make_volume(w2)
    ids2, vol2_c = scan.compact(vol2)
    g2 = Graph.build(vol2).upload(0)
    b2 = synth.make_boxes(w2)
    _case(g2, vol2_c, len(ids2), b2, "second graph")
    _case(g, vol_c, S, boxes[:400], "first graph again")
    g2.close()
    g.close()


def test_noalloc_rejects_batches_beyond_the_scratch():
    """More boxes than the scratch has 20-byte slots for: MG_ELIMIT from the host-side check,
    before anything is enqueued (the buffers are still sized for the whole batch)."""
    w = synth.workload(1, n_boxes=10)
    vol = synth.make_volume(w)
    g = Graph.build(vol).upload(0)
    n = (64 << 20) // 20 + 1
    boxes = torch.zeros((n, 6), dtype=torch.int32, device="cuda")
    out = torch.empty((n, g.info()["nseg"]), dtype=torch.float32, device="cuda")
    with pytest.raises(MGError) as e:
        g.query_noalloc(boxes, out=out)
    assert e.value.code == -8 and "scratch" in str(e.value)
    torch.cuda.synchronize()
    g.close()
