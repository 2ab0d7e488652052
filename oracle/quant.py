"""Scalar quantization of interpolation weights and error propagation.

ORACLE (test infrastructure only). Follows the paper's description in plain
Python / NumPy fp64:

- Sec. "Compression": the open range (0, 1) is divided into 2^b equal bins;
  each bin is represented by one codeword, and the empirical standard deviation
  of the weights that fall into the bin is kept with it. Readings taken here:
  the codeword is the mean of the bin's weights (the value that represents them
  best in the least-squares sense), the standard deviation is the population
  one, and a bin no weight falls into gets its midpoint and the standard
  deviation of a uniform distribution over the bin.
- Table "bitstream" (C): each codeword and each standard deviation is stored
  with 20 bits. Reading: a codeword is the nearest multiple of 2^-20 inside
  (0, 1), a standard deviation the nearest multiple of sigma_max / (2^20 - 1),
  where sigma_max (header field 4, 32 bits) is the largest one in fp32; the
  quantizer's codebook is the stored one.
- Sec. "Implementation Details": a lerp (i, j, w) equals (j, i, 1 - w); both w
  and 1 - w are quantized and the orientation with the smaller quantization
  error is kept (ties: w).
- Nodes whose predecessors and quantized weight coincide are the same node
  (re-use, Sec. "Compression"); a lerp of a node with itself is that node.
- Sec. "Error Propagation", Eq. (error): component i of (1 - w) a + w b carries
  dmu_i = mu_i sqrt((da_i / a_i)^2 + (db_i / b_i)^2 + 2 (dw / w)^2); sources are
  certain. Reading: a term whose component is absent from that child (a_i = 0)
  contributes zero.
- A box's uncertainty: the count scattered onto each node n is c_n (cubes of
  n times 8^level); per segment the node terms add in quadrature,
  d_count_s = sqrt(sum_n (c_n dmu_n[s])^2) (the sum rule of the same section
  applied to the per-node products c_n mu_n, with c_n exact).
"""
from __future__ import annotations

import math

import numpy as np


CODE_BITS = 20


def codebook(weights, bits: int):
    """(codeword [2^bits], sigma [2^bits]) learned from weights in (0, 1), at the stored resolution."""
    B = 1 << bits
    w = np.asarray(weights, dtype=np.float64)
    k = np.minimum((w * B).astype(np.int64), B - 1)
    mean = np.empty(B)
    sd = np.empty(B)
    for b in range(B):
        sel = w[k == b]
        if len(sel):
            mean[b] = sel.mean()
            sd[b] = math.sqrt(float(((sel - sel.mean()) ** 2).mean()))
        else:
            mean[b] = (b + 0.5) / B
            sd[b] = 1.0 / B / math.sqrt(12.0)
    scale = float(1 << CODE_BITS)
    code = np.array([min(max(math.floor(m * scale + 0.5), 1), scale - 1) / scale for m in mean])
    smax = float(np.float32(sd.max()))
    top = float((1 << CODE_BITS) - 1)
    sig = np.array([float(np.float32(smax * min(math.floor(x / smax * top + 0.5), top) / top)) if smax > 0 else 0.0
                    for x in sd])
    return code, sig


def quantize_dag(nseg: int, a, b, w, bits: int):
    """Quantize the DAG whose internal nodes n = nseg + k are (1 - w[k]) a[k] + w[k] b[k], given
    children-first. Returns (rep, nodes, code, sig): rep[n] = index of node n's representative in
    `nodes`, a list of (first, second, weight, sigma) for the quantized internal nodes (indices
    >= nseg, in creation order; weights are float32 codewords, stored <= 1/2)."""
    code, sig = codebook(w, bits)
    code32 = code.astype(np.float32)
    B = 1 << bits
    n_int = len(a)
    rep = list(range(nseg)) + [0] * n_int
    made = {}
    nodes = []
    for k in range(n_int):
        x, y = rep[a[k]], rep[b[k]]
        if x == y:
            rep[nseg + k] = x
            continue
        wk = float(w[k])
        k1 = min(int(wk * B), B - 1)
        k2 = min(int((1.0 - wk) * B), B - 1)
        flip = abs((1.0 - wk) - float(code32[k2])) < abs(wk - float(code32[k1]))
        kb = k2 if flip else k1
        first, second = (y, x) if flip else (x, y)
        c = np.float32(code32[kb])
        if c > np.float32(0.5):
            first, second, c = second, first, np.float32(1.0) - c
        key = (first, second, float(c))
        if key in made:
            rep[nseg + k] = made[key]
            continue
        idx = nseg + len(nodes)
        made[key] = idx
        rep[nseg + k] = idx
        nodes.append((first, second, float(c), float(np.float32(sig[kb]))))
    return rep, nodes, code32, sig.astype(np.float32)


def propagate(nseg: int, nodes):
    """Dense fp64 (mu [N, nseg], dmu [N, nseg]) for sources 0..nseg-1 and the quantized nodes."""
    N = nseg + len(nodes)
    mu = np.zeros((N, nseg))
    dmu = np.zeros((N, nseg))
    mu[np.arange(nseg), np.arange(nseg)] = 1.0
    for j, (x, y, c, s) in enumerate(nodes):
        n = nseg + j
        mu[n] = (1.0 - c) * mu[x] + c * mu[y]
        with np.errstate(divide="ignore", invalid="ignore"):
            ra = np.where(mu[x] > 0, dmu[x] / mu[x], 0.0)
            rb = np.where(mu[y] > 0, dmu[y] / mu[y], 0.0)
        dmu[n] = mu[n] * np.sqrt(ra * ra + rb * rb + 2.0 * (s / c) ** 2)
    return mu, dmu


def box_histogram(node_counts: dict, mu, dmu, volume: float):
    """(fractions [nseg], uncertainties [nseg]) of a box from {node: voxel count scattered onto it}."""
    f = np.zeros(mu.shape[1])
    var = np.zeros(mu.shape[1])
    for n, c in node_counts.items():
        f += c * mu[n]
        var += (c * dmu[n]) ** 2
    return f / volume, np.sqrt(var) / volume
