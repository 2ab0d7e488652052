"""Continuous-batching server for box-histogram requests on one GPU.

Requests (a box, optionally with one RGBA8 transfer function) arrive over
time. The server keeps the graph resident and owns a fixed set of slots; a
slot is a HIP stream with its own device buffers (boxes, results, workspace,
transfer functions) sized for `max_batch` requests. Whenever a slot is free
and requests are waiting, the waiting requests (up to `max_batch`) are
admitted as one batch on that slot: boxes are copied to the device, the
batched query kernels run (replayed from a captured HIP graph when graphs are
enabled), transfer-function requests of the batch are propagated together,
and results are copied back into pinned host memory. Batches on different
slots overlap on the device, so requests that arrive while others are in
flight are admitted as soon as a slot frees up. A request completes when its
batch's completion event has fired; its latency is completion time minus
arrival time.

Admission is bounded by a device-memory budget: the number of slots (and, if
one full slot does not fit, the batch size) is reduced until the slots fit the
budget, so a small budget makes requests wait longer instead of failing.

Admission is also size-aware: the host counts each box's footprint cubes in
closed form, and a box of at least `split_cubes` cubes is cut into sub-boxes
along its longest axis at aligned positions (multiples of a power of two, so
few cubes are cut) that are answered as separate rows of the same batch, in
parallel on different workgroups. Histograms of disjoint parts add up, so the
request's row is the volume-weighted sum of its rows' fractions (in fp64).
"""
from __future__ import annotations

import gc
import time
from collections import deque
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

from ._lib import check
from .graph import Graph, _torch


@dataclass
class ServeStats:
    latency_s: np.ndarray            # per request, completion - arrival
    completion_s: np.ndarray         # per request, relative to the start
    batches: int
    batch_sizes: List[int] = field(default_factory=list)
    wall_s: float = 0.0

    def summary(self) -> dict:
        lat = self.latency_s * 1e3
        return {
            "requests": int(len(lat)), "batches": self.batches,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "qps": float(len(lat) / self.wall_s) if self.wall_s > 0 else 0.0,
        }


def cube_counts(boxes: np.ndarray, dims) -> np.ndarray:
    """Footprint cubes of each box (uint32 [n, 6] rows x0, y0, z0, dx, dy, dz, clipped to dims),
    in closed form per level: the aligned cells of the level inside the box minus those covered
    by cells of the next level."""
    b = np.asarray(boxes, dtype=np.int64)
    d = np.asarray(dims, dtype=np.int64)
    lo = np.minimum(b[:, :3], d)
    hi = np.minimum(b[:, :3] + b[:, 3:], d)
    out = np.zeros(len(b), dtype=np.int64)
    l = 0
    while True:
        one = 1 << l
        a, c = (lo + one - 1) >> l, hi >> l
        outer = np.prod(np.maximum(c - a, 0), axis=1)
        if not outer.any():
            break
        pa, pc = (lo + 2 * one - 1) >> (l + 1), hi >> (l + 1)
        inner = np.prod(np.maximum(2 * (pc - pa), 0), axis=1)
        out += outer - inner
        l += 1
    return out


def split_box(box, dims, pieces: int):
    """Sub-boxes (uint32 [m, 6]) covering the clipped box, cut along its longest axis into about
    `pieces` parts at multiples of a power of two."""
    lo = [min(int(box[a]), int(dims[a])) for a in range(3)]
    hi = [min(int(box[a]) + int(box[3 + a]), int(dims[a])) for a in range(3)]
    ext = [h - l for l, h in zip(lo, hi)]
    ax = int(np.argmax(ext))
    if pieces < 2 or ext[ax] < 2 or min(ext) == 0:
        return np.array([list(lo) + ext], dtype=np.uint32)
    align = 1 << max(0, int(np.floor(np.log2(ext[ax] / pieces))))
    cuts = list(range((lo[ax] // align + 1) * align, hi[ax], align))
    edges = [lo[ax]] + cuts + [hi[ax]]
    out = []
    for a, b in zip(edges[:-1], edges[1:]):
        r = list(lo) + ext
        r[ax], r[3 + ax] = a, b - a
        out.append(r)
    return np.array(out, dtype=np.uint32)


class _Slot:
    def __init__(self, g: Graph, max_batch: int, max_tf: int, device, use_graphs: bool, classes):
        torch = _torch()
        inf = g.info()
        self.S, self.N = inf["nseg"], inf["n_nodes"]
        self.max_batch = max_batch
        self.stream = torch.cuda.Stream(device=device)
        self.h_boxes = torch.zeros((max_batch, 6), dtype=torch.int32, pin_memory=True)
        self.d_boxes = torch.zeros((max_batch, 6), dtype=torch.int32, device=device)
        self.d_out = torch.zeros((max_batch, self.S), dtype=torch.float32, device=device)
        self.h_out = torch.zeros((max_batch, self.S), dtype=torch.float32, pin_memory=True)
        self.max_tf = max_tf
        if max_tf:
            self.h_tf = torch.zeros((max_tf, self.S, 4), dtype=torch.uint8, pin_memory=True)
            self.d_tf = torch.zeros((max_tf, self.S, 4), dtype=torch.uint8, device=device)
            self.d_pal = torch.zeros((max_tf, self.N, 4), dtype=torch.float32, device=device)
        nbytes = g.workspace_bytes(max_batch)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        check(g._lib.mg_workspace_init(g._h, self.ws.data_ptr(), nbytes, self.stream.cuda_stream))
        self.event = torch.cuda.Event()
        self.busy = False
        self.reqs = None
        self.n_rows = 0
        self.graphs = {}
        self.classes = [c for c in classes if c <= max_batch] or [max_batch]
        if use_graphs:
            self._capture(g)

    def _capture(self, g: Graph):
        torch = _torch()
        for c in self.classes:
            # warm up the launch path outside capture (fills the library's launch caches)
            with torch.cuda.stream(self.stream):
                g.query(self.d_boxes[:c], out=self.d_out[:c], workspace=self.ws, stream=self.stream)
            self.stream.synchronize()
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=self.stream):
                g.query(self.d_boxes[:c], out=self.d_out[:c], workspace=self.ws, stream=self.stream)
            self.graphs[c] = graph
        # the first replay of a captured graph pays its one-time upload, and the first launch of the
        # propagation kernels their loading: do both here, not while serving
        with torch.cuda.stream(self.stream):
            for c in self.classes:
                self.graphs[c].replay()
            if self.max_tf:
                g.propagate_tf(self.d_tf[:1], out=self.d_pal[:1], stream=self.stream)
        self.stream.synchronize()

    def size_class(self, k: int) -> int:
        for c in self.classes:
            if k <= c:
                return c
        return self.classes[-1]

    def launch(self, g: Graph, boxes: np.ndarray, tfs: Optional[np.ndarray]):
        """Enqueue one batch: H2D boxes, query (graph replay or direct), TF propagation, D2H results."""
        torch = _torch()
        k = len(boxes)
        use = self.size_class(k) if self.graphs else k
        hb = self.h_boxes.numpy()
        hb[:k] = boxes.view(np.int32)
        if use > k:
            hb[k:use] = 0   # empty boxes pad the captured size
        with torch.cuda.stream(self.stream):
            self.d_boxes[:use].copy_(self.h_boxes[:use], non_blocking=True)
            if self.graphs:
                self.graphs[use].replay()
            else:
                g.query(self.d_boxes[:k], out=self.d_out[:k], workspace=self.ws, stream=self.stream)
            if tfs is not None and len(tfs):
                t = len(tfs)
                self.h_tf.numpy()[:t] = tfs
                self.d_tf[:t].copy_(self.h_tf[:t], non_blocking=True)
                g.propagate_tf(self.d_tf[:t], out=self.d_pal[:t], stream=self.stream)
            self.h_out[:k].copy_(self.d_out[:k], non_blocking=True)
            self.event.record(self.stream)
        self.busy = True


class Server:
    """Slots of HIP streams serving box-histogram requests with continuous batching."""

    def __init__(self, g: Graph, slots: int = 4, max_batch: int = 4096, max_tf: int = 64,
                 budget_bytes: Optional[int] = None, use_graphs: bool = True,
                 classes=(64, 256, 1024, 4096, 16384), split_cubes: int = 1 << 18,
                 piece_cubes: int = 1 << 16):
        torch = _torch()
        self.g = g
        inf = g.info()
        S, N = inf["nseg"], inf["n_nodes"]
        self.dims = inf["dims"][0]
        self.split_cubes, self.piece_cubes = split_cubes, piece_cubes

        def slot_bytes(b, t):
            return g.workspace_bytes(b) + b * (24 + 4 * S) + t * (4 * S + 16 * N)

        if budget_bytes is not None:
            # fewer slots first, then smaller batches and fewer TFs per batch
            while slots > 1 and slots * slot_bytes(max_batch, max_tf) > budget_bytes:
                slots -= 1
            while max_batch > 1 and slot_bytes(max_batch, max_tf) > budget_bytes:
                max_batch //= 2
                max_tf = min(max_tf, max_batch)
            while max_tf > 1 and slot_bytes(max_batch, max_tf) > budget_bytes:
                max_tf //= 2
            if slot_bytes(max_batch, max_tf) > budget_bytes:
                raise ValueError("device-memory budget %d B cannot hold one request (needs %d B)"
                                 % (budget_bytes, slot_bytes(max_batch, max_tf)))
        self.max_batch, self.max_tf = max_batch, max_tf
        device = torch.device("cuda:%d" % g._device)
        self.slots = [_Slot(g, max_batch, max_tf, device, use_graphs, classes) for _ in range(slots)]
        self.device_bytes = slots * slot_bytes(max_batch, max_tf)

    def serve(self, boxes: np.ndarray, arrivals: np.ndarray, tf_index: Optional[np.ndarray] = None,
              tfs: Optional[np.ndarray] = None, results: Optional[np.ndarray] = None) -> ServeStats:
        """Serve requests i = 0..n-1 arriving at arrivals[i] seconds after the start.

        tf_index[i] >= 0 makes request i also propagate tfs[tf_index[i]] ([S, 4] uint8).
        Results (fp32 [n, S]) are written into `results` if given. Python's cyclic garbage
        collector is paused while serving (a full collection can stall the loop for milliseconds)."""
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._serve(boxes, arrivals, tf_index, tfs, results)
        finally:
            if was_enabled:
                gc.enable()

    def _serve(self, boxes, arrivals, tf_index, tfs, results) -> ServeStats:
        n = len(boxes)
        boxes = np.ascontiguousarray(boxes, dtype=np.uint32)
        arrivals = np.asarray(arrivals, dtype=np.float64)
        assert n == len(arrivals) and np.all(np.diff(arrivals) >= 0), "arrivals must be sorted"
        done = np.full(n, np.nan)
        # rows of each request: the box itself, or its sub-boxes
        cubes = cube_counts(boxes, self.dims)
        rows = {}
        for i in np.nonzero(cubes >= self.split_cubes)[0]:
            sub = split_box(boxes[i], self.dims, int(min(64, -(-cubes[i] // self.piece_cubes))))
            if len(sub) > 1 and len(sub) <= self.max_batch:
                rows[int(i)] = sub
        pending = deque()
        nxt = 0
        batches, sizes = 0, []
        finished = 0
        t0 = time.perf_counter()
        while finished < n:
            now = time.perf_counter() - t0
            while nxt < n and arrivals[nxt] <= now:
                pending.append(nxt)
                nxt += 1
            progressed = False
            for sl in self.slots:
                if sl.busy and sl.event.query():
                    r = sl.reqs
                    h = sl.h_out[:sl.n_rows].numpy()
                    row = 0
                    for i in r.tolist():
                        sub = rows.get(i)
                        if sub is None:
                            if results is not None:
                                results[i] = h[row]
                            row += 1
                        else:  # volume-weighted sum of the sub-boxes' fractions
                            v = np.prod(sub[:, 3:].astype(np.float64), axis=1)
                            comb = (h[row:row + len(sub)].astype(np.float64).T @ v) / v.sum()
                            if results is not None:
                                results[i] = comb
                            row += len(sub)
                    done[r] = time.perf_counter() - t0
                    finished += len(r)
                    sl.busy = False
                    progressed = True
            for sl in self.slots:
                if not pending:
                    break
                if sl.busy:
                    continue
                # requests whose rows fit max_batch, of which at most max_tf carry a transfer function
                take, n_tf, n_rows = [], 0, 0
                while pending:
                    i = pending[0]
                    k_i = len(rows[i]) if i in rows else 1
                    if n_rows + k_i > self.max_batch:
                        break
                    if tf_index is not None and tf_index[i] >= 0:
                        if n_tf == self.max_tf:
                            break
                        n_tf += 1
                    take.append(pending.popleft())
                    n_rows += k_i
                r = np.array(take, dtype=np.int64)
                k = len(r)
                tf_batch = None
                if n_tf:
                    sel = tf_index[r]
                    tf_batch = tfs[sel[sel >= 0]]
                sl.reqs = r
                sl.n_rows = n_rows
                bx = boxes[r] if not any(i in rows for i in take) else np.concatenate(
                    [rows[i] if i in rows else boxes[i:i + 1] for i in take])
                sl.launch(self.g, bx, tf_batch)
                batches += 1
                sizes.append(k)
                progressed = True
            if not progressed and not pending and nxt < n:
                wait = arrivals[nxt] - (time.perf_counter() - t0)
                if wait > 200e-6:
                    time.sleep(wait - 100e-6)
        wall = time.perf_counter() - t0
        return ServeStats(latency_s=done - arrivals, completion_s=done, batches=batches, batch_sizes=sizes,
                          wall_s=wall)
