"""Binary-lerp DAG semantics: forward expansion, reverse push, topological levels.

ORACLE (test infrastructure only). A graph is given as plain arrays: nodes
``0 .. nseg-1`` are sources (node s stands for the unit vector of segment s);
every other node n is the linear interpolation ``(1 - w_n) * node[a_n] +
w_n * node[b_n]`` of two earlier-defined nodes (Sec. "Factorization": each
internal node mixes exactly two predecessors with edge weights summing to 1;
Figs. "factorization", "tree", "DAG").

- ``expand_exact``  every node's mixture over the segments with exact
                    rational weights (Python ``Fraction``).
- ``expand_fp64``   the same in fp64, dense.
- ``forward``       a value per source carried to every node by the same
                    interpolations (colour propagation, Sec. "Reconstruction").
- ``push``          the transpose: mass placed on nodes flows down to the
                    sources, each node splitting its mass (1-w, w) between its
                    two predecessors, in reverse topological order.
- ``levels``        topological level: 0 for sources, otherwise one more than
                    the larger level of the two predecessors (Sec.
                    "Reconstruction").
- ``defer_window``  the steps a node may run in: from its level to one less
                    than the smallest level of its successors (Sec.
                    "Reconstruction", deferred evaluation, Fig. "dagtopo").

Topological order is found here by depth-first search; nothing assumes that
node IDs are sorted.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _topo_order(nseg: int, a, b):
    """Internal nodes ordered so that both predecessors come first (iterative DFS)."""
    n_nodes = nseg + len(a)
    state = np.zeros(n_nodes, dtype=np.int8)  # 0 new, 1 on stack, 2 done
    state[:nseg] = 2
    order = []
    for root in range(nseg, n_nodes):
        if state[root] == 2:
            continue
        stack = [(root, 0)]
        while stack:
            n, k = stack.pop()
            if k == 0:
                if state[n] == 2:
                    continue
                if state[n] == 1:
                    raise ValueError("cycle at node %d" % n)
                state[n] = 1
            kids = (int(a[n - nseg]), int(b[n - nseg]))
            if k < 2:
                stack.append((n, k + 1))
                c = kids[k]
                if not (0 <= c < n_nodes):
                    raise ValueError("node %d has out-of-range predecessor %d" % (n, c))
                if state[c] == 1:
                    raise ValueError("cycle through node %d" % c)
                if state[c] == 0:
                    stack.append((c, 0))
            else:
                state[n] = 2
                order.append(n)
    return order


def expand_exact(nseg: int, a, b, wnum, wden):
    """List of {segment: Fraction} for every node; internal weights w_n = wnum/wden (weight of b)."""
    mix = [{s: Fraction(1)} for s in range(nseg)] + [None] * len(a)
    for n in _topo_order(nseg, a, b):
        i = n - nseg
        w = Fraction(int(wnum[i]), int(wden[i]))
        out = {}
        for s, v in mix[int(a[i])].items():
            out[s] = out.get(s, Fraction(0)) + (1 - w) * v
        for s, v in mix[int(b[i])].items():
            out[s] = out.get(s, Fraction(0)) + w * v
        mix[n] = {s: v for s, v in out.items() if v != 0}
    return mix


def expand_fp64(nseg: int, a, b, w) -> np.ndarray:
    """Dense fp64 [n_nodes, nseg] node mixtures."""
    eye = np.eye(nseg, dtype=np.float64)
    return forward(nseg, a, b, w, eye)


def forward(nseg: int, a, b, w, src_values: np.ndarray) -> np.ndarray:
    """fp64 [n_nodes, C]: source values carried to every node, v_n = (1-w_n) v_a + w_n v_b."""
    src = np.asarray(src_values, dtype=np.float64)
    out = np.zeros((nseg + len(a),) + src.shape[1:], dtype=np.float64)
    out[:nseg] = src
    for n in _topo_order(nseg, a, b):
        i = n - nseg
        wi = float(w[i])
        out[n] = (1.0 - wi) * out[int(a[i])] + wi * out[int(b[i])]
    return out


def push(nseg: int, a, b, w, node_mass) -> np.ndarray:
    """fp64 [nseg]: mass on nodes pushed down to the sources (reverse topological order)."""
    m = np.array(node_mass, dtype=np.float64, copy=True)
    for n in reversed(_topo_order(nseg, a, b)):
        i = n - nseg
        if m[n] == 0.0:
            continue
        wi = float(w[i])
        m[int(a[i])] += (1.0 - wi) * m[n]
        m[int(b[i])] += wi * m[n]
        m[n] = 0.0
    return m[:nseg]


def levels(nseg: int, a, b) -> np.ndarray:
    lv = np.zeros(nseg + len(a), dtype=np.int64)
    for n in _topo_order(nseg, a, b):
        i = n - nseg
        lv[n] = max(lv[int(a[i])], lv[int(b[i])]) + 1
    return lv


def defer_window(nseg: int, a, b):
    """(first, last) step of every node: its level, and one less than its lowest successor's level.

    Nodes without successors (sinks) get last = depth of the graph."""
    lv = levels(nseg, a, b)
    depth = int(lv.max()) if len(lv) else 0
    lo_succ = np.full(len(lv), depth + 1, dtype=np.int64)
    for i in range(len(a)):
        n = nseg + i
        for c in (int(a[i]), int(b[i])):
            lo_succ[c] = min(lo_succ[c], lv[n])
    return lv, lo_succ - 1
