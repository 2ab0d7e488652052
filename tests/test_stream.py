"""Bit-packed graph stream (Sec. "Compression", Table "bitstream"): the library's mg_pack / mg_unpack
against the stream oracle (oracle/stream.py) and the quantization oracle (oracle/quant.py).

Pins of the oracle that do not come from its own code: a two-voxel stream whose every field is
derived by hand from the paper's table; the closed-form length; and a parse of the library's stream
that must describe, mip voxel by mip voxel, the mixtures the quantization oracle computes on its own.
"""
import math
import struct

import numpy as np
import pytest

from oracle import quant, stream
from paper_2009_02702_amd import Graph, MGError, synth


def _assemble(flds):
    acc, pos = 0, 0
    for v, w in flds:
        acc |= v << pos
        pos += w
    return acc.to_bytes((pos + 7) // 8, "little"), pos


def test_two_voxel_stream_field_by_field():
    """Volume x = (5, 9): sources 0 (label 5) and 1 (label 9); level 1 holds one voxel, the node
    (0.5, 0.5) = (1 - 1/2) e0 + 1/2 e1. One quantizer bit: bin 1 = [1/2, 1) holds the weight 1/2
    (codeword 1/2, sigma 0); bin 0 is empty (midpoint 1/4, sigma (1/2)/sqrt(12) = sigma_max)."""
    g = Graph.build(np.array([[[5, 9]]], dtype=np.uint32))
    q = g.quantize(1)
    smax = float(np.float32(0.5 / math.sqrt(12.0)))
    smax_bits = struct.unpack("<I", struct.pack("<f", smax))[0]
    hand = [
        (2, 32), (0, 1), (2 - 1, 6), (smax_bits, 32),      # (1) sources (2) integer input (3) 2 bits/node (4)
        (2, 32), (1, 32), (1, 32), (1 - 1, 4), (1, 2),      # (5) 2x1x1 (6) 1 bit (7) one internal node
        (1, 2), (0, 2),                                     # level 0: r = 1, i_min = 0
        (0, 2), (2, 2),                                     # level 1: r = 0 (one node ID), i_min = 2
        (0, 1), (1, 1),                                     # (A) level 0 voxels; level 1 needs no bits
        (0, 2), (1, 2), (1, 1),                             # (B) node 2 = (first 0, second 1, bin 1)
        (2 ** 18, 20), (2 ** 20 - 1, 20),                   # (C) bin 0: 1/4, sigma_max
        (2 ** 19, 20), (0, 20),                             #     bin 1: 1/2, 0
        (5, 32), (9, 32),                                   # labels of the sources
    ]
    want, nbits = _assemble(hand)
    assert nbits == 332 and len(want) == 42
    assert q.pack() == want
    assert stream.write(2, (2, 1, 1), 1, [[0, 1], [2]], [(0, 1, 1)], [0.25, 0.5], [smax, 0.0], [5, 9]) == want
    f = stream.read(want)
    assert f["nodes"] == [(0, 1, 1)] and f["labels"] == [5, 9] and f["level_table"] == [(1, 0), (0, 2)]
    u = Graph.unpack(want)
    assert np.array_equal(u.export_map(1), np.array([[[2]]], dtype=np.uint32))
    assert u.export_dag()["alpha"][2] == np.float32(0.5) and list(u.segment_ids()) == [5, 9]


def _quantized(config, dims, segments, bits):
    w = synth.workload(config, dims=dims, segments=segments)
    vol = synth.make_volume(w)
    g = Graph.build(vol)
    return vol, g, g.quantize(bits)


def _expected_fields(q):
    """Stream fields of a library graph, from its exported arrays."""
    inf = q.info()
    S, N, L = inf["nseg"], inf["n_nodes"], inf["n_levels"]
    d = q.export_dag()
    cw, sg, _, nc = q.export_codebook(with_code=True)
    nodes = []
    for n in range(S, N):
        k = int(nc[n])
        same = d["alpha"][n] == cw[k]
        a, b = int(d["child_a"][n]), int(d["child_b"][n])
        nodes.append((a, b, k) if same else (b, a, k))
    levels = [q.export_map(l).ravel() for l in range(L)]
    return S, tuple(inf["dims"][0]), inf["quant_bits"], levels, nodes, cw, sg, q.segment_ids()


@pytest.mark.parametrize("config,dims,segments,bits", [
    (2, (30, 26, 22), 25, 5), (4, (28, 20, 18), 16, 9), (1, (17, 9, 5), 6, 3), (2, (40, 1, 33), 40, 16)])
def test_library_stream_equals_the_oracle_stream(config, dims, segments, bits):
    _, _, q = _quantized(config, dims, segments, bits)
    S, dm, b, levels, nodes, cw, sg, labels = _expected_fields(q)
    data = q.pack()
    assert data == stream.write(S, dm, b, levels, nodes, cw, sg, labels)
    f = stream.read(data)
    N = S + len(nodes)
    assert f["bits_per_node"] == max(1, math.ceil(math.log2(N))) and f["n_internal"] == len(nodes)
    for (r, lo), ids in zip(f["level_table"], levels):
        assert lo == int(ids.min()) and r == math.ceil(math.log2(int(ids.max()) - lo + 1))
    sizes = [len(ids) for ids in levels]
    nbits = stream.size_bits(S, len(nodes), b, sizes, [r for r, _ in f["level_table"]])
    assert f["bits_used"] == nbits and len(data) == (nbits + 7) // 8
    assert f["code"] == [float(c) for c in cw] and f["sigma"] == [float(s) for s in sg]


def test_stream_describes_the_oracle_quantized_mixtures():
    """Parse the library's stream, rebuild every mip voxel's mixture from the parsed nodes and
    codebook, and compare with the quantization oracle's mixture of the same voxel (computed from
    the exact graph by the oracle alone)."""
    vol, g, q = _quantized(2, (36, 30, 26), 30, 6)
    S = g.info()["nseg"]
    d = g.export_dag()
    rep, onodes, _, _ = quant.quantize_dag(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:] / d["wden"][S:], 6)
    mu_o, _ = quant.propagate(S, onodes)
    f = stream.read(q.pack())
    pnodes = []
    for a, b, k in f["nodes"]:
        c = f["code"][k]
        pnodes.append((a, b, c, 0.0) if c <= 0.5 else (b, a, float(np.float32(1.0) - np.float32(c)), 0.0))
    mu_s, _ = quant.propagate(S, pnodes)
    for l in range(g.info()["n_levels"]):
        exact = g.export_map(l).ravel()
        packed = f["levels"][l]
        for i in range(0, len(exact), 3):
            assert np.allclose(mu_s[packed[i]], mu_o[rep[int(exact[i])]], rtol=0, atol=1e-12), (l, i)


def test_unpack_of_pack_is_the_same_graph():
    _, _, q = _quantized(2, (30, 26, 22), 25, 7)
    u = Graph.unpack(q.pack())
    a, b = q.info(), u.info()
    for k in ("nseg", "n_nodes", "depth", "n_levels", "quant_bits", "dims"):
        assert a[k] == b[k], k
    da, db = q.export_dag(), u.export_dag()
    for k in ("child_a", "child_b", "alpha", "wnum", "wden"):
        assert np.array_equal(da[k], db[k]), k
    for l in range(a["n_levels"]):
        assert np.array_equal(q.export_map(l), u.export_map(l))
    for x, y in zip(q.export_codebook(with_code=True), u.export_codebook(with_code=True)):
        assert np.array_equal(x, y)
    assert np.array_equal(q.segment_ids(), u.segment_ids())
    assert u.pack() == q.pack()
    q.lut_build()
    u.lut_build()
    for x, y in zip(q.export_lut(with_err=True), u.export_lut(with_err=True)):
        assert np.array_equal(x, y)


def test_save_and_load_keep_the_codebook(tmp_path):
    _, _, q = _quantized(4, (28, 20, 18), 16, 8)
    p = str(tmp_path / "q.mg")
    q.save(p)
    r = Graph.load(p)
    assert r.info()["quant_bits"] == 8
    for x, y in zip(q.export_codebook(with_code=True), r.export_codebook(with_code=True)):
        assert np.array_equal(x, y)
    assert r.pack() == q.pack()


def test_stream_errors():
    vol, g, q = _quantized(1, (12, 10, 8), 5, 4)
    with pytest.raises(MGError) as e:
        g.pack()                                            # exact weights: nothing to index
    assert e.value.code == -4
    data = q.pack()
    for cut in (1, 5, 20, len(data) // 2, len(data) - 5):
        with pytest.raises(MGError) as e:
            Graph.unpack(data[:cut])
        assert e.value.code == -7, cut
    flds = stream.fields(*_expected_fields(q))
    bad = list(flds)
    bad[1] = (1, 1)                                          # fractional input
    with pytest.raises(MGError):
        Graph.unpack(stream.assemble(bad))
    bad = list(flds)
    bad[2] = (bad[2][0] + 1, 6)                              # bits per node do not match the node count
    with pytest.raises(MGError):
        Graph.unpack(stream.assemble(bad))
    # the first internal node refers to itself: its triple follows 9 header fields, 2 per level and
    # one field per mip voxel
    inf = q.info()
    S, L = inf["nseg"], inf["n_levels"]
    i = 9 + 2 * L + sum(int(np.prod(inf["dims"][l])) for l in range(L))
    bpn = flds[2][0] + 1
    assert flds[i][1] == bpn and flds[i + 2][1] == 4
    bad = list(flds)
    bad[i] = (S, bpn)
    with pytest.raises(MGError) as e:
        Graph.unpack(stream.assemble(bad))
    assert e.value.code == -7
