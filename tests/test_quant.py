"""Scalar-quantized weights and propagated uncertainty (Sec. "Compression", Sec. "Implementation
Details", Sec. "Error Propagation" Eq. (error)): the oracle pinned to closed forms, and the library's
quantized graph and lookup table checked against the oracle on the CPU."""
import math

import numpy as np

from oracle import dag, footprint, quant, scan
from paper_2009_02702_amd import Graph, MGError, synth


def test_codebook_is_the_mean_and_spread_of_each_bin():
    w = np.array([0.1, 0.12, 0.3, 0.31, 0.33])
    code, sig = quant.codebook(w, 2)                      # bins [0, .25) [.25, .5) [.5, .75) [.75, 1)
    m = (0.3 + 0.31 + 0.33) / 3
    q = 2.0 ** -20                                        # stored resolution of codewords
    assert np.abs(code[:2] - [0.11, m]).max() <= q / 2 and (code * 2 ** 20 == np.round(code * 2 ** 20)).all()
    s1 = math.sqrt(((0.3 - m) ** 2 + (0.31 - m) ** 2 + (0.33 - m) ** 2) / 3)
    smax = 0.25 / math.sqrt(12)                           # the empty bins' spread is the largest
    assert np.allclose(sig, [0.01, s1, smax, smax], rtol=0, atol=smax / (2 ** 20 - 1))
    assert np.allclose(code[2:], [0.625, 0.875])


def test_symmetric_orientation_keeps_the_smaller_error():
    # same predecessors and same bin: one node (re-use)
    rep, nodes, code, _ = quant.quantize_dag(2, [0, 0], [1, 1], [0.26, 0.49], 2)
    assert len(nodes) == 1 and rep[2] == rep[3] == 2
    assert nodes[0][:2] == (0, 1) and nodes[0][2] == float(np.float32(code[1]))
    # a codebook learned from {0.2, 0.3, 0.7} with 2 bins: codewords 0.25 and 0.7 (to 2^-20). For
    # w = 0.3, |0.3 - 0.25| = 0.05 > |(1 - 0.3) - 0.7| ~ 0: the flipped orientation (1, 0, 0.7) is kept
    # and stored with the weight <= 1/2 as (0, 1, 1 - 0.7); for w = 0.2 (error 0.05 vs 0.1) w is kept.
    code, _ = quant.codebook([0.2, 0.3, 0.7], 1)
    assert np.allclose(code, [0.25, 0.7], rtol=0, atol=2.0 ** -21)
    rep, nodes, code32, _ = quant.quantize_dag(2, [0, 0, 0], [1, 1, 1], [0.2, 0.3, 0.7], 1)
    c07 = float(np.float32(1) - np.float32(code[1]))
    tri = {n: nodes[rep[n] - 2][:3] for n in (2, 3, 4)}
    assert tri[2] == (0, 1, float(np.float32(0.25)))   # w = 0.2: kept
    assert tri[3] == (0, 1, c07)                         # w = 0.3: flipped, 0.7 e0 + 0.3 e1 as before
    assert tri[4] == (1, 0, c07)                         # w = 0.7 = 0.3 e0 + 0.7 e1: its mirror


def test_degenerate_lerp_collapses_to_its_predecessor():
    # two internal nodes that quantize to the same node, and a third mixing them: (1 - w) x + w x = x
    rep, nodes, _, _ = quant.quantize_dag(2, [0, 0, 2], [1, 1, 3], [0.3, 0.31, 0.5], 2)
    assert len(nodes) == 1 and rep[2] == rep[3] == rep[4] == 2


def test_rank1_uncertainty_closed_form():
    """Sources are certain, so a rank-1 node (1 - w) e_a + w e_b has dmu = mu sqrt(2) sigma / w."""
    nodes = [(0, 1, 0.25, 0.01)]
    mu, dmu = quant.propagate(2, nodes)
    assert np.allclose(mu[2], [0.75, 0.25])
    r = math.sqrt(2) * 0.01 / 0.25
    assert np.allclose(dmu[2], [0.75 * r, 0.25 * r])
    # (1 - 0.5) node2 + 0.5 e_0 with sigma 0.02: component 0 has a = 0.75 (relative r) and b = 1
    # (certain); component 1 has a = 0.25 (relative r) and no b term
    nodes.append((2, 0, 0.5, 0.02))
    mu, dmu = quant.propagate(2, nodes)
    assert np.allclose(mu[3], [0.5 * 0.75 + 0.5, 0.5 * 0.25])
    rw = 0.02 / 0.5
    assert np.allclose(dmu[3], mu[3] * math.sqrt(r * r + 2 * rw * rw))


def _exact(shape, nseg, seed):
    vol = np.random.default_rng(seed).integers(0, nseg, size=shape).astype(np.uint32)
    g = Graph.build(vol)
    S = g.info()["nseg"]
    d = g.export_dag()
    w = (d["wnum"][S:] / d["wden"][S:]).astype(np.float64)
    return vol, g, S, d, w


def test_library_quantizer_matches_the_oracle():
    """Same merges (node count), same quantized mixture and uncertainty for every mip voxel."""
    for w_ in (synth.workload(2, dims=(30, 26, 22), segments=25), synth.workload(4, dims=(28, 20, 18), segments=16)):
        vol = synth.make_volume(w_)
        g = Graph.build(vol)
        S = g.info()["nseg"]
        d = g.export_dag()
        wts = d["wnum"][S:] / d["wden"][S:]
        for bits in (2, 5, 9):
            rep, nodes, code, sig = quant.quantize_dag(S, d["child_a"][S:], d["child_b"][S:], wts, bits)
            q = g.quantize(bits)
            assert q.info()["n_nodes"] == S + len(nodes), bits
            cw, sg, _ = q.export_codebook()
            assert np.array_equal(cw, code) and np.allclose(sg, sig, rtol=1e-5, atol=1e-9)
            mu, dmu = quant.propagate(S, nodes)
            q.lut_build()
            ptr, seg, val, err = q.export_lut(with_err=True)
            for l in range(1, g.info()["n_levels"]):
                me, mq = g.export_map(l).ravel(), q.export_map(l).ravel()
                for ne, nq in zip(me[::7], mq[::7]):
                    row = slice(int(ptr[nq]), int(ptr[nq + 1]))
                    o = rep[int(ne)]
                    want = mu[o][seg[row]]
                    assert np.allclose(val[row], want, rtol=1e-6, atol=1e-7)
                    assert np.allclose(err[row], dmu[o][seg[row]], rtol=1e-4, atol=1e-9)
                    assert np.count_nonzero(mu[o]) == len(seg[row])


def test_quantized_rows_stay_convex_and_fine_bits_are_near_exact():
    vol, g, S, d, w = _exact((16, 14, 12), 12, 7)
    q = g.quantize(16)
    q.lut_build()
    g.lut_build()
    p, s_, v = q.export_lut()
    assert q.info()["n_nodes"] == g.info()["n_nodes"]
    for n in range(q.info()["n_nodes"]):
        assert abs(float(v[int(p[n]):int(p[n + 1])].astype(np.float64).sum()) - 1.0) < 1e-6
    q3 = g.quantize(3)
    q3.lut_build()
    p, s_, v = q3.export_lut()
    for n in range(q3.info()["n_nodes"]):
        assert abs(float(v[int(p[n]):int(p[n + 1])].astype(np.float64).sum()) - 1.0) < 1e-6
    assert q3.info()["n_nodes"] < g.info()["n_nodes"]
    with np.testing.assert_raises(MGError):
        q3.quantize(4)
    with np.testing.assert_raises(MGError):
        g.quantize(0)
    with np.testing.assert_raises(MGError):
        g.quantize(17)
    with np.testing.assert_raises(MGError):
        g.export_codebook()


def test_quantized_box_error_at_nine_bits_is_within_the_paper_bound():
    """Queries with 512-bin weights: the paper reports errors of about 0.3% and at most 0.5% (Sec.
    "Fast Sub-Volume Queries"). On a synthetic Voronoi volume, every segment fraction of random boxes
    stays within 0.5% of the exact one (O1), and the propagated uncertainty covers the typical error."""
    w_ = synth.workload(2, dims=(48, 44, 40), segments=40, n_boxes=150)
    vol = synth.make_volume(w_)
    g = Graph.build(vol)
    S = g.info()["nseg"]
    d = g.export_dag()
    rep, nodes, _, _ = quant.quantize_dag(S, d["child_a"][S:], d["child_b"][S:], d["wnum"][S:] / d["wden"][S:], 9)
    mu, dmu = quant.propagate(S, nodes)
    ids, vol_c = scan.compact(vol)
    boxes = synth.make_boxes(w_)
    _, ref = scan.box_counts(vol_c, S, boxes)
    maps = [g.export_map(l) for l in range(g.info()["n_levels"])]
    dims = vol.shape[::-1]
    worst, errs, unc = 0.0, [], []
    for i, bx in enumerate(boxes.astype(int)):
        counts = {}
        for lev, c in footprint.assembly(bx[:3], bx[3:], dims):
            n = rep[int(maps[lev][c[2], c[1], c[0]])]
            counts[n] = counts.get(n, 0) + 8 ** lev
        vol_b = np.prod(np.minimum(bx[:3] + bx[3:], dims) - bx[:3])
        if vol_b <= 0:
            continue
        f, u = quant.box_histogram(counts, mu, dmu, float(vol_b))
        worst = max(worst, float(np.abs(f - ref[i]).max()))
        nz = ref[i] > 0
        errs.append(np.abs(f - ref[i])[nz])
        unc.append(u[nz])
        assert abs(f.sum() - 1.0) < 1e-9                       # unbiased: fractions sum to 1
    assert worst <= 0.005, worst
    e, u = np.concatenate(errs), np.concatenate(unc)
    assert np.median(e) <= np.median(u) * 3 + 1e-12
