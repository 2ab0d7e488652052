"""Continuous-batching server for box-histogram requests on one GPU.

Requests (a box, optionally with one RGBA8 transfer function) arrive over
time. The server keeps the graph resident and owns a fixed set of slots; a
slot is a HIP stream with its own device buffers (boxes, results, workspace,
transfer functions) sized for `max_batch` requests. Whenever a slot is free
and requests are waiting, the waiting requests (up to `max_batch`) are
admitted as one batch on that slot: boxes are copied to the device, the
batched query kernels run (replayed from a captured HIP graph when graphs are
enabled), transfer-function requests of the batch are propagated together,
each transfer-function request's box is coloured with its propagated
palette (mg_box_colour: the box's mean colour from its footprint cubes), and
results are copied back into pinned host memory. Batches on different
slots overlap on the device, so requests that arrive while others are in
flight are admitted as soon as a slot frees up. A request completes when its
batch's completion event has fired; its latency is completion time minus
arrival time.

Admission is bounded by a device-memory budget: the number of slots (and, if
one full slot does not fit, the batch size) is reduced until the slots fit the
budget, so a small budget makes requests wait longer instead of failing.

Admission is also size-aware: the host counts each box's footprint cubes in
closed form, and a box of at least `split_cubes` cubes is cut into up to
`max_pieces` sub-boxes of about `piece_cubes` cubes
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


TRACE_FIELDS = ("t_admit", "t_launched", "t_seen", "device_ms", "oldest_arrival", "requests", "rows", "tfs",
                "max_cubes", "slot", "h2d_ms", "query_ms", "tf_ms", "d2h_ms")


@dataclass
class ServeStats:
    latency_s: np.ndarray            # per request, completion - arrival
    completion_s: np.ndarray         # per request, relative to the start
    batches: int
    batch_sizes: List[int] = field(default_factory=list)
    wall_s: float = 0.0
    # per batch (seconds from the start unless stated): admission, return of the launch calls,
    # completion seen by the loop, device time between the batch's first and last stream event,
    # arrival of its oldest request, requests, rows, transfer functions, largest box (cubes), slot,
    # and the host time (ms) spent enqueuing each step: boxes copy, query, TF work, results copy
    trace: Optional[np.ndarray] = None

    def summary(self) -> dict:
        lat = self.latency_s * 1e3
        out = {
            "requests": int(len(lat)), "batches": self.batches,
            "mean_batch": float(np.mean(self.batch_sizes)) if self.batch_sizes else 0.0,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "max_ms": float(lat.max()), "qps": float(len(lat) / self.wall_s) if self.wall_s > 0 else 0.0,
        }
        if self.trace is not None and len(self.trace):
            tr = self.trace
            wait = (tr[:, 0] - tr[:, 4]) * 1e3                 # oldest request's wait before admission
            launch = (tr[:, 1] - tr[:, 0]) * 1e3               # host time in the launch calls
            seen = (tr[:, 2] - tr[:, 1]) * 1e3                 # launch return -> completion seen
            worst = int(np.argmax(tr[:, 2] - tr[:, 4]))
            out["batch_ms"] = {
                "admit_wait_p99": float(np.percentile(wait, 99)), "launch_p99": float(np.percentile(launch, 99)),
                "launch_max": float(launch.max()), "device_p99": float(np.percentile(tr[:, 3], 99)),
                "device_max": float(tr[:, 3].max()), "launch_to_seen_p99": float(np.percentile(seen, 99)),
                "worst_batch": {k: float(tr[worst, i]) for i, k in enumerate(TRACE_FIELDS)},
            }
        return out


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
            # per row: the palette its box is coloured with (0xFFFFFFFF: none), and the colour
            self.h_pal_of = torch.zeros(max_batch, dtype=torch.int32, pin_memory=True)
            self.d_pal_of = torch.zeros(max_batch, dtype=torch.int32, device=device)
            self.d_col = torch.zeros((max_batch, 4), dtype=torch.float32, device=device)
            self.h_col = torch.zeros((max_batch, 4), dtype=torch.float32, pin_memory=True)
        nbytes = g.workspace_bytes(max_batch)
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        check(g._lib.mg_workspace_init(g._h, self.ws.data_ptr(), nbytes, self.stream.cuda_stream))
        self.event = torch.cuda.Event(enable_timing=True)
        self.event0 = torch.cuda.Event(enable_timing=True)
        self.busy = False
        self.n_tf = 0
        self.trace = None
        self.reqs = None
        self.n_rows = 0
        self.graphs = {}
        # every batch size up to max_batch has a class: max_batch itself is always one
        self.classes = sorted({int(c) for c in classes if c < max_batch} | {int(max_batch)})
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
                self.d_pal_of.fill_(-1)
                g.box_colour(self.d_pal[:1], self.d_boxes[:1], self.d_pal_of[:1], out=self.d_col[:1],
                             stream=self.stream)
        self.stream.synchronize()

    def size_class(self, k: int) -> int:
        """The smallest captured batch size that holds k rows (k <= max_batch)."""
        if not 0 < k <= self.max_batch:
            raise ValueError("batch of %d rows for a slot of %d" % (k, self.max_batch))
        for c in self.classes:
            if k <= c:
                return c
        raise AssertionError("max_batch is always a class")

    def launch(self, g: Graph, boxes: np.ndarray, tfs: Optional[np.ndarray],
               pal_of_row: Optional[np.ndarray] = None):
        """Enqueue one batch: H2D boxes, query (graph replay or direct), TF propagation and the
        colour of each TF request's box, D2H results. pal_of_row[r] is the TF (index into tfs)
        row r is coloured with, or -1."""
        torch = _torch()
        k = len(boxes)
        use = self.size_class(k) if self.graphs else k
        if use < k:
            raise AssertionError("size class below the batch")
        hb = self.h_boxes.numpy()
        hb[:k] = boxes.view(np.int32)
        if use > k:
            hb[k:use] = 0   # empty boxes pad the captured size
        self.n_tf = 0
        clock = time.perf_counter
        with torch.cuda.stream(self.stream):
            c0 = clock()
            self.event0.record(self.stream)
            self.d_boxes[:use].copy_(self.h_boxes[:use], non_blocking=True)
            c1 = clock()
            if self.graphs:
                self.graphs[use].replay()
            else:
                g.query(self.d_boxes[:k], out=self.d_out[:k], workspace=self.ws, stream=self.stream)
            c2 = clock()
            if tfs is not None and len(tfs):
                t = len(tfs)
                if t > self.max_tf:
                    raise ValueError("%d transfer functions for a slot of %d" % (t, self.max_tf))
                self.h_tf.numpy()[:t] = tfs
                self.d_tf[:t].copy_(self.h_tf[:t], non_blocking=True)
                g.propagate_tf(self.d_tf[:t], out=self.d_pal[:t], stream=self.stream)
                self.h_pal_of.numpy()[:k] = pal_of_row
                self.d_pal_of[:k].copy_(self.h_pal_of[:k], non_blocking=True)
                g.box_colour(self.d_pal[:t], self.d_boxes[:k], self.d_pal_of[:k], out=self.d_col[:k],
                             stream=self.stream)
                self.h_col[:k].copy_(self.d_col[:k], non_blocking=True)
                self.n_tf = t
            c3 = clock()
            self.h_out[:k].copy_(self.d_out[:k], non_blocking=True)
            self.event.record(self.stream)
            c4 = clock()
        self.busy = True
        return [1e3 * (c1 - c0), 1e3 * (c2 - c1), 1e3 * (c3 - c2), 1e3 * (c4 - c3)]


class Server:
    """Slots of HIP streams serving box-histogram requests with continuous batching."""

    def __init__(self, g: Graph, slots: int = 4, max_batch: int = 4096, max_tf: int = 64,
                 budget_bytes: Optional[int] = None, use_graphs: bool = True,
                 classes=(64, 256, 1024, 4096, 16384), split_cubes: int = 1 << 18,
                 piece_cubes: int = 1 << 15, max_pieces: int = 128):
        torch = _torch()
        self.g = g
        inf = g.info()
        S, N = inf["nseg"], inf["n_nodes"]
        self.dims = inf["dims"][0]
        self.split_cubes, self.piece_cubes, self.max_pieces = split_cubes, piece_cubes, max_pieces

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
        self.warm()

    def warm(self, rounds: int = 3) -> None:
        """Every slot busy at once with a full batch of empty boxes, every TF slot used and
        every copy, `rounds` times: the runtime's per-launch resources are sized for the heaviest
        load before the first request (a host stall of several ms in a copy or graph launch
        otherwise shows up once a run, as the load first grows)."""
        torch = _torch()
        empty = np.zeros((self.max_batch, 6), dtype=np.uint32)
        S = self.g.info()["nseg"]
        tfs = np.zeros((self.max_tf, S, 4), dtype=np.uint8) if self.max_tf else None
        pal = np.zeros(self.max_batch, dtype=np.int32) if self.max_tf else None
        for _ in range(rounds):
            for sl in self.slots:
                sl.launch(self.g, empty, tfs, pal)
            for sl in self.slots:
                sl.event.synchronize()
                sl.busy = False
        torch.cuda.synchronize()

    def serve(self, boxes: np.ndarray, arrivals: np.ndarray, tf_index: Optional[np.ndarray] = None,
              tfs: Optional[np.ndarray] = None, results: Optional[np.ndarray] = None,
              colours: Optional[np.ndarray] = None) -> ServeStats:
        """Serve requests i = 0..n-1 arriving at arrivals[i] seconds after the start.

        tf_index[i] >= 0 makes request i also propagate tfs[tf_index[i]] ([S, 4] uint8) and
        colour its box with the result: colours[i] (fp32 [n, 4], if given) receives the box's
        mean colour under that transfer function (rows of other requests are left alone).
        Results (fp32 [n, S]) are written into `results` if given. Python's cyclic garbage
        collector is paused while serving (a full collection can stall the loop for milliseconds)."""
        if tf_index is not None and (np.asarray(tf_index) >= 0).any():
            if self.max_tf == 0:
                raise ValueError("transfer-function requests need a server with max_tf > 0")
            if tfs is None:
                raise ValueError("tf_index given without tfs")
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._serve(boxes, arrivals, tf_index, tfs, results, colours)
        finally:
            if was_enabled:
                gc.enable()

    def _admit(self, pending, rows, tf_index):
        """Requests from the head of the queue for one batch: their rows fit max_batch and at most
        max_tf of them carry a transfer function. Returns (requests, rows, TF requests)."""
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
        return take, n_rows, n_tf

    def _serve(self, boxes, arrivals, tf_index, tfs, results, colours) -> ServeStats:
        n = len(boxes)
        boxes = np.ascontiguousarray(boxes, dtype=np.uint32)
        arrivals = np.asarray(arrivals, dtype=np.float64)
        assert n == len(arrivals) and np.all(np.diff(arrivals) >= 0), "arrivals must be sorted"
        done = np.full(n, np.nan)
        # rows of each request: the box itself, or its sub-boxes
        cubes = cube_counts(boxes, self.dims)
        rows = {}
        for i in np.nonzero(cubes >= self.split_cubes)[0]:
            sub = split_box(boxes[i], self.dims, int(min(self.max_pieces, -(-cubes[i] // self.piece_cubes))))
            if len(sub) > 1 and len(sub) <= self.max_batch:
                rows[int(i)] = sub
        pending = deque()
        nxt = 0
        batches, sizes = 0, []
        trace = []
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
                    t_seen = time.perf_counter() - t0
                    r = sl.reqs
                    h = sl.h_out[:sl.n_rows].numpy()
                    hc = sl.h_col[:sl.n_rows].numpy() if sl.n_tf else None
                    row = 0
                    for i in r.tolist():
                        sub = rows.get(i)
                        k_i = 1 if sub is None else len(sub)
                        if sub is None:
                            if results is not None:
                                results[i] = h[row]
                            if hc is not None and colours is not None and tf_index[i] >= 0:
                                colours[i] = hc[row]
                        else:  # volume-weighted sums of the sub-boxes' fractions and colours
                            v = np.prod(sub[:, 3:].astype(np.float64), axis=1)
                            if results is not None:
                                results[i] = (h[row:row + k_i].astype(np.float64).T @ v) / v.sum()
                            if hc is not None and colours is not None and tf_index[i] >= 0:
                                colours[i] = (hc[row:row + k_i].astype(np.float64).T @ v) / v.sum()
                        row += k_i
                    done[r] = t_seen
                    sl.trace[2] = t_seen
                    sl.trace[3] = sl.event0.elapsed_time(sl.event)
                    trace.append(sl.trace)
                    finished += len(r)
                    sl.busy = False
                    progressed = True
            for sl in self.slots:
                if not pending:
                    break
                if sl.busy:
                    continue
                t_admit = time.perf_counter() - t0
                take, n_rows, n_tf = self._admit(pending, rows, tf_index)
                if not take:
                    break   # the head request fits no batch (cannot happen: max_batch, max_tf >= 1)
                r = np.array(take, dtype=np.int64)
                k = len(r)
                tf_batch = pal_of_row = None
                split = any(i in rows for i in take)
                if n_tf:
                    sel = tf_index[r]
                    tf_batch = tfs[sel[sel >= 0]]
                    # position of each TF request's transfer function in tf_batch, per row
                    t_of_req = np.full(k, -1, dtype=np.int32)
                    t_of_req[sel >= 0] = np.arange(n_tf, dtype=np.int32)
                    pal_of_row = t_of_req if not split else np.repeat(
                        t_of_req, [len(rows[i]) if i in rows else 1 for i in take])
                sl.reqs = r
                sl.n_rows = n_rows
                bx = boxes[r] if not split else np.concatenate(
                    [rows[i] if i in rows else boxes[i:i + 1] for i in take])
                steps = sl.launch(self.g, bx, tf_batch, pal_of_row)
                t_launched = time.perf_counter() - t0
                sl.trace = [t_admit, t_launched, 0.0, 0.0, float(arrivals[take[0]]), k, n_rows, n_tf,
                            float(cubes[r].max()), float(self.slots.index(sl))] + steps
                batches += 1
                sizes.append(k)
                progressed = True
            if not progressed and not pending and nxt < n:
                wait = arrivals[nxt] - (time.perf_counter() - t0)
                if wait > 200e-6:
                    time.sleep(wait - 100e-6)
        wall = time.perf_counter() - t0
        return ServeStats(latency_s=done - arrivals, completion_s=done, batches=batches, batch_sizes=sizes,
                          wall_s=wall, trace=np.array(trace, dtype=np.float64).reshape(-1, len(TRACE_FIELDS)))
