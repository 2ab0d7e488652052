"""Bit-packed graph stream (Sec. "Compression", Table "bitstream"): writer and reader.

ORACLE (test infrastructure only): plain Python integers as bit strings, field by field in the
table's order. Readings taken here (the paper gives widths and order, not the bit convention):

- every field is an unsigned integer written least significant bit first; bit i of the stream is
  bit (i mod 8) of byte i // 8; zero bits pad the last byte;
- (3) holds bits-per-node minus 1 (range [1, 64] in 6 bits), (6) the bit rate minus 1 ([1, 16]
  in 4 bits); bits per node = ceil(log2(#nodes)), at least 1;
- (4) sigma_max is the IEEE fp32 bit pattern; (C) stores per bin the codeword times 2^20 and
  sigma / sigma_max times (2^20 - 1), 20 bits each, the weight first;
- (B) per internal node, in ID order: (first, second, bin) meaning (1 - code) first + code second;
- an addition after (C): the input label of each source, 32 bits (the paper's sources are the
  input IDs; here sources are the distinct labels numbered in increasing order);
- the number of levels follows from the resolution (halving, rounding up, until 1^3).
"""
from __future__ import annotations

import math
import struct

import numpy as np

CODE_BITS = 20


def ceil_log2(v: int) -> int:
    """Smallest r with 2^r >= v (v >= 1)."""
    r = 0
    while (1 << r) < v:
        r += 1
    return r


def level_shapes(dims):
    """[(X, Y, Z)] per level: halve with rounding up until 1^3."""
    d = list(dims)
    out = [tuple(d)]
    while max(d) > 1:
        d = [(x + 1) // 2 for x in d]
        out.append(tuple(d))
    return out


def fields(S, dims, bits, levels, nodes, code, sigma, labels):
    """The stream as a list of (value, width), in order.

    levels: per level a flat sequence of node IDs (x fastest); nodes: per internal node (first,
    second, bin); code / sigma: fp32 codewords (multiples of 2^-20) and sigmas per bin."""
    N = S + len(nodes)
    bpn = max(1, ceil_log2(N))
    smax = float(np.float32(max(sigma)))
    out = [(S, 32), (0, 1), (bpn - 1, 6), (struct.unpack("<I", struct.pack("<f", smax))[0], 32)]
    out += [(int(dims[0]), 32), (int(dims[1]), 32), (int(dims[2]), 32), (bits - 1, 4), (len(nodes), bpn)]
    lo_r = []
    for ids in levels:
        lo, hi = int(min(ids)), int(max(ids))
        lo_r.append((lo, ceil_log2(hi - lo + 1)))
        out += [(ceil_log2(hi - lo + 1), bpn), (lo, bpn)]
    for ids, (lo, r) in zip(levels, lo_r):
        out += [(int(i) - lo, r) for i in ids]
    for a, b, k in nodes:
        out += [(int(a), bpn), (int(b), bpn), (int(k), bits)]
    top = (1 << CODE_BITS) - 1
    for c, s in zip(code, sigma):
        m = float(c) * (1 << CODE_BITS)
        assert m == math.floor(m) and 0 < m < (1 << CODE_BITS)
        out += [(int(m), CODE_BITS), (min(math.floor(float(s) / smax * top + 0.5), top) if smax > 0 else 0, CODE_BITS)]
    out += [(int(l), 32) for l in labels]
    return out


def assemble(flds) -> bytes:
    """Concatenate (value, width) fields least significant bit first."""
    acc, pos = 0, 0
    for v, w in flds:
        assert 0 <= v < (1 << w) or (w == 0 and v == 0), (v, w)
        acc |= v << pos
        pos += w
    return acc.to_bytes((pos + 7) // 8, "little")


def write(S, dims, bits, levels, nodes, code, sigma, labels) -> bytes:
    return assemble(fields(S, dims, bits, levels, nodes, code, sigma, labels))


class _Reader:
    def __init__(self, data: bytes):
        self.v = int.from_bytes(data, "little")
        self.n = 8 * len(data)
        self.pos = 0

    def get(self, w: int) -> int:
        if self.pos + w > self.n:
            raise ValueError("truncated stream")
        x = (self.v >> self.pos) & ((1 << w) - 1)
        self.pos += w
        return x


def read(data: bytes) -> dict:
    """Parse a stream into its fields (levels as flat node-ID arrays, x fastest)."""
    rd = _Reader(data)
    S = rd.get(32)
    frac = rd.get(1)
    bpn = rd.get(6) + 1
    smax = struct.unpack("<f", struct.pack("<I", rd.get(32)))[0]
    dims = (rd.get(32), rd.get(32), rd.get(32))
    bits = rd.get(4) + 1
    n_int = rd.get(bpn)
    shapes = level_shapes(dims)
    table = [(rd.get(bpn), rd.get(bpn)) for _ in shapes]          # (r, i_min)
    levels = []
    for (r, lo), (X, Y, Z) in zip(table, shapes):
        levels.append(np.array([lo + rd.get(r) for _ in range(X * Y * Z)], dtype=np.int64))
    nodes = [(rd.get(bpn), rd.get(bpn), rd.get(bits)) for _ in range(n_int)]
    top = (1 << CODE_BITS) - 1
    code, sigma = [], []
    for _ in range(1 << bits):
        code.append(rd.get(CODE_BITS) / float(1 << CODE_BITS))
        sigma.append(float(np.float32(smax * rd.get(CODE_BITS) / top)))
    labels = [rd.get(32) for _ in range(S)]
    return {"S": S, "fractional": frac, "bits_per_node": bpn, "sigma_max": smax, "dims": dims, "bits": bits,
            "n_internal": n_int, "level_table": table, "levels": levels, "nodes": nodes, "code": code,
            "sigma": sigma, "labels": labels, "bits_used": rd.pos}


def size_bits(S, n_int, bits, level_sizes, level_r) -> int:
    """Closed form of the stream length in bits (before the byte padding)."""
    bpn = max(1, ceil_log2(S + n_int))
    return (32 + 1 + 6 + 32 + 96 + 4 + bpn + 2 * bpn * len(level_sizes) + sum(n * r for n, r in zip(level_sizes, level_r))
            + n_int * (2 * bpn + bits) + (1 << bits) * 2 * CODE_BITS + 32 * S)
