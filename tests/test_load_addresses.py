"""The query kernels' load addresses, replayed on the host (no GPU).

mg_check_load_addresses builds each box's slabs with the kernels' own slab builder and walks
them with the kernels' own tile-walk helpers (and, for slabs summed from row runs, the kernels'
own segment enumeration) (2^ltx units x 2^(6-ltx) rows per load, UNROLL
loads per block, every load issued, consumed or not), then checks every lane load: inside its
slab, inside the map buffer (the 32-bit maps of both orientations, or the 16-bit level-0 copies),
and for consumed loads the element of a footprint cube of the box; every cube of the footprint is
read once (the count equals the closed-form cube count). The naive scan's loads over the whole
box are replayed the same way. Run over the bench batch, the full-size volumes (far corners,
where byte offsets pass 4 GiB), odd row parities, widest rows and tiny volumes.
"""
import ctypes

import numpy as np
import pytest

from paper_2009_02702_amd import _lib, synth


def _check(dims, boxes, use16, unroll, naive=True, runs=False, run_min=0):
    """runs: slabs with rows of at least run_min cubes (0: the library default) from row runs."""
    lib = _lib.load()
    b = np.ascontiguousarray(boxes, dtype=np.uint32).reshape(-1, 6)
    counts = (ctypes.c_uint64 * 4)()
    flags = int(use16) | (2 if naive else 0) | (4 if runs else 0) | (run_min << 8)
    rc = lib.mg_check_load_addresses(int(dims[0]), int(dims[1]), int(dims[2]), flags,
                                     b.ctypes.data_as(ctypes.c_void_p), len(b), int(unroll), counts)
    msg = lib.mg_last_error().decode() if rc else ""
    assert rc == 0, "%s use16=%d unroll=%d runs=%d/%d: %s" % (dims, use16, unroll, runs, run_min, msg)
    return list(counts)


def _far_corner_boxes(dims):
    X, Y, Z = dims
    out = []
    for e in (1, 2, 3, 5, 8, 17, 64, 100, 255, 256, 513, 1024, 4096):
        ex, ey, ez = min(e, X), min(e, Y), min(e, Z)
        out.append([X - ex, Y - ey, Z - ez, ex, ey, ez])
    out += [[0, 0, 0, X, Y, Z], [X - 1, 0, 0, 1, Y, Z], [0, Y - 1, 0, X, 1, Z], [0, 0, Z - 1, X, Y, 1],
            [X - 37 if X > 37 else 0, Y - 41 if Y > 41 else 0, 0, 37, 41, Z], [X - 3, 0, Z - 7 if Z > 7 else 0, 13, Y, 12]]
    return np.array(out, dtype=np.int64).clip(0).astype(np.uint32)


def _odd_parity_boxes(dims, n, seed):
    """Boxes whose every corner coordinate is odd or even at random, extents 1..300."""
    rng = np.random.default_rng(seed)
    d = np.asarray(dims)
    lo = rng.integers(0, d, size=(n, 3))
    ext = rng.integers(1, 301, size=(n, 3))
    return np.concatenate([lo, ext], axis=1).astype(np.uint32)


def test_bench_batch_every_load():
    """All 100,000 boxes of the 512^3 bench batch, 16-bit level 0, the default unroll; then with
    rows of 16 cubes or more read from row runs."""
    w = synth.workload(2)
    boxes = synth.make_boxes(w)
    counts = _check(w.dims, boxes, 1, 16, naive=False)
    assert counts[0] == len(boxes) and counts[3] > 2.5e9
    for run_min, share in ((0, 0.5), (1, 0.1)):
        runs = _check(w.dims, boxes, 1, 16, naive=False, runs=True, run_min=run_min)
        assert runs[0] == counts[0] and runs[1] == counts[1] and runs[3] == counts[3]
        assert runs[2] < counts[2] * share   # fewer loads and segment walks than lane loads


@pytest.mark.parametrize("config", [1, 3, 4, 5])
def test_full_size_volumes_sampled(config):
    """Query loads of sampled, far-corner and odd-parity boxes; naive-scan loads of the far-corner
    boxes up to 100^3 and of small odd-parity boxes."""
    w = synth.workload(config)
    far = _far_corner_boxes(w.dims)
    boxes = np.concatenate([synth.make_boxes(w, 800), far, _odd_parity_boxes(w.dims, 200, config)])
    small = np.concatenate([far[:7], _odd_parity_boxes(w.dims, 100, config + 10) % np.uint32(64) + 1])
    small[len(far[:7]):, :3] = _odd_parity_boxes(w.dims, 100, config + 10)[:, :3]
    for use16, unroll, runs, rm in ((1, 8, False, 0), (0, 16, False, 0), (1, 4, False, 0), (1, 8, True, 0),
                                    (0, 4, True, 1), (1, 16, True, 16)):
        _check(w.dims, boxes, use16, unroll, naive=False, runs=runs, run_min=rm)
        _check(w.dims, small, use16, unroll, naive=True, runs=runs, run_min=rm)


def test_widest_rows_and_largest_units():
    """Rows of 32,768 cubes (16,384 pairs), slabs of 2^24 units, the last voxel of the volume."""
    dims = (32768, 1024, 2)
    boxes = [[0, 0, 0, 32768, 1024, 2], [1, 3, 0, 32767, 5, 2], [32767, 1023, 1, 1, 1, 1],
             [5, 0, 0, 32000, 1, 1], [0, 1, 1, 32768, 1023, 1]]
    for use16, unroll, runs, rm in ((1, 8, False, 0), (0, 4, False, 0), (1, 16, False, 0), (1, 8, True, 0),
                                    (1, 4, True, 1)):
        _check(dims, boxes, use16, unroll, runs=runs, run_min=rm)


@pytest.mark.parametrize("dims", [(1, 1, 1), (2, 3, 5), (7, 1, 9), (5, 8, 3), (1, 13, 2)])
def test_tiny_volumes_every_box(dims):
    X, Y, Z = dims
    rng = [[(a, b - a) for a in range(D) for b in range(a + 1, D + 1)] for D in dims]
    boxes = [[x0, y0, z0, dx, dy, dz] for x0, dx in rng[0] for y0, dy in rng[1] for z0, dz in rng[2]]
    boxes += [[X, 0, 0, 1, 1, 1], [0, 0, 0, 0, 1, 1], [0, 0, 0, 0xFFFFFFFF, 0xFFFFFFFF, 0xFFFFFFFF]]
    for use16, runs in ((0, False), (1, False), (1, True)):
        counts = _check(dims, boxes, use16, 4, runs=runs, run_min=1)
        assert counts[0] == len(boxes) - 2     # the two empty boxes are skipped


def test_rejects_bad_arguments():
    lib = _lib.load()
    counts = (ctypes.c_uint64 * 4)()
    b = np.zeros((1, 6), dtype=np.uint32)
    p = b.ctypes.data_as(ctypes.c_void_p)
    assert lib.mg_check_load_addresses(8, 8, 8, 1, p, 1, 3, counts) == -1
    assert lib.mg_check_load_addresses(0, 8, 8, 1, p, 1, 8, counts) == -1
    assert lib.mg_check_load_addresses(8, 8, 8, 1, p, 1, 8, None) == -1
    assert lib.mg_check_load_addresses(8, 8, 8, 8, p, 1, 8, counts) == -1
    assert lib.mg_check_load_addresses(8, 8, 8, 0x80, p, 1, 8, counts) == -1
