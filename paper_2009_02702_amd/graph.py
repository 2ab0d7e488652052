"""Python binding of the Mixture Graph library: the same calls as include/mg.h.

Host arrays are NumPy; device buffers are torch tensors (PyTorch provides
device memory and streams only). Query and propagation calls enqueue HIP
kernels on the current torch stream and return without synchronising.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np

from . import _lib
from ._lib import BuildOpts, Info, LaunchCfg, check

VARIANTS = ("batched", "plain", "naive")
FACTORIZERS = {"halving": 0, "reduction": 1, "occurrence": 2}


def _torch():
    import torch
    return torch


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dptr(t) -> ctypes.c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


class Graph:
    """A Mixture Graph built on the CPU and, after upload(), resident on one GPU."""

    def __init__(self, handle: ctypes.c_void_p):
        self._h = handle
        self._lib = _lib.load()
        self._ws = None
        self._ws_boxes = 0
        self._bound = None   # caller-owned device buffer of mg_bind_device, kept alive here

    # -------------------------------------------------------------- construction
    @classmethod
    def build(cls, volume: np.ndarray, defer: bool = True, max_depth: int = 0, threads: int = 0,
              factorizer: str = "halving", tau: int = 3) -> "Graph":
        """mg_build on a (nz, ny, nx) ID volume; uint8/uint16 volumes are widened to uint32.
        factorizer: "halving", or the paper's greedy "reduction" (phi2) / "occurrence" (phi1) with cutoff tau."""
        vol = np.asarray(volume)
        if vol.ndim != 3:
            raise ValueError("volume must be 3-D (nz, ny, nx)")
        if vol.dtype != np.uint32:
            if vol.dtype.kind not in "ui" or (vol.size and int(vol.min()) < 0):
                raise ValueError("volume must hold non-negative integer IDs")
            vol = vol.astype(np.uint32)
        vol = np.ascontiguousarray(vol)
        nz, ny, nx = vol.shape
        o = BuildOpts(nx=nx, ny=ny, nz=nz, defer=1 if defer else 0, max_depth=max_depth, threads=threads,
                      factorizer=FACTORIZERS[factorizer], tau=tau)
        h = ctypes.c_void_p()
        check(_lib.load().mg_build(vol.ctypes.data_as(ctypes.c_void_p), ctypes.byref(o), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def load(cls, path: str) -> "Graph":
        h = ctypes.c_void_p()
        check(_lib.load().mg_load(path.encode(), ctypes.byref(h)))
        return cls(h)

    def save(self, path: str) -> None:
        check(self._lib.mg_save(self._h, path.encode()))

    def pack(self) -> bytes:
        """The bit-packed graph stream (mg_pack) of a quantized graph."""
        size = ctypes.c_uint64()
        check(self._lib.mg_pack(self._h, None, 0, ctypes.byref(size)))
        buf = (ctypes.c_uint8 * max(size.value, 1))()
        check(self._lib.mg_pack(self._h, buf, size.value, ctypes.byref(size)))
        return bytes(buf)[:size.value]

    @classmethod
    def unpack(cls, stream: bytes, threads: int = 0) -> "Graph":
        """A host graph from a bit-packed stream (mg_unpack)."""
        h = ctypes.c_void_p()
        data = bytes(stream)
        check(_lib.load().mg_unpack(data, len(data), threads, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def unpack_device(cls, stream: bytes, device: int = 0, threads: int = 0) -> "Graph":
        """mg_unpack_device: a graph on `device` from a bit-packed stream, its voxel IDs decoded on
        the GPU."""
        h = ctypes.c_void_p()
        data = bytes(stream)
        check(_lib.load().mg_unpack_device(data, len(data), threads, int(device), ctypes.byref(h)))
        g = cls(h)
        g._device = int(device)
        return g

    def close(self) -> None:
        if self._h:
            self._ws = None
            self._lib.mg_free(self._h)
            self._h = None
            self._bound = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -------------------------------------------------------------- host views
    def info(self) -> dict:
        i = Info()
        check(self._lib.mg_info(self._h, ctypes.byref(i)))
        return {
            "nseg": i.nseg, "n_nodes": i.n_nodes, "depth": i.depth, "n_levels": i.n_levels,
            "dims": [tuple(i.dims[l]) for l in range(i.n_levels)], "map_voxels": i.map_voxels,
            "device_bytes": i.device_bytes, "device": i.device, "max_mixture": i.max_mixture,
            "quant_bits": i.quant_bits, "runs_mask": i.runs_mask,
        }

    def export_dag(self) -> dict:
        inf = self.info()
        n, d = inf["n_nodes"], inf["depth"]
        spec = (("child_a", np.uint32, n), ("child_b", np.uint32, n), ("alpha", np.float32, n),
                ("wnum", np.uint64, n), ("wden", np.uint64, n), ("rank", np.uint32, n),
                ("rank_ptr", np.uint32, d + 2), ("step", np.uint32, n), ("sched", np.uint32, n),
                ("step_ptr", np.uint32, d + 2))
        out = {k: np.zeros(m, dtype=t) for k, t, m in spec}
        check(self._lib.mg_export_dag(self._h, *[out[k].ctypes.data_as(ctypes.c_void_p) for k, _, _ in spec]))
        return out

    def export_map(self, level: int) -> np.ndarray:
        nx, ny, nz = self.info()["dims"][level]
        out = np.zeros((nz, ny, nx), dtype=np.uint32)
        check(self._lib.mg_export_map(self._h, level, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def segment_ids(self) -> np.ndarray:
        out = np.zeros(self.info()["nseg"], dtype=np.uint32)
        check(self._lib.mg_segment_ids(self._h, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    # -------------------------------------------------------------- device
    def upload(self, device: int = 0) -> "Graph":
        check(self._lib.mg_upload(self._h, int(device)))
        self._device = int(device)
        self._bound = None
        self._ws = None
        return self

    def device_bytes(self) -> int:
        """Bytes of the one device buffer mg_bind_device fills."""
        b = ctypes.c_uint64()
        check(self._lib.mg_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def bind(self, buffer, stream=None) -> "Graph":
        """mg_bind_device: the graph's device arrays in a caller-owned torch tensor (uint8, at least
        device_bytes() bytes, on the GPU the graph will run on). The tensor is kept referenced here
        for as long as the graph is bound."""
        if not buffer.is_cuda or not buffer.is_contiguous():
            raise ValueError("buffer must be a contiguous device tensor")
        nbytes = buffer.numel() * buffer.element_size()
        check(self._lib.mg_bind_device(self._h, int(buffer.device.index or 0), _dptr(buffer), nbytes,
                                       _stream_ptr(stream)))
        self._device = int(buffer.device.index or 0)
        self._bound = buffer
        self._ws = None
        return self

    def nnz_bound(self, boxes, out=None, stream=None):
        """mg_query_nnz_bound: int32 [n] upper bound on each box's non-zero segments."""
        torch = _torch()
        if boxes.dim() != 2 or boxes.shape[1] != 6 or boxes.element_size() != 4:
            raise ValueError("boxes must be a 32-bit [n, 6] tensor")
        n = boxes.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=boxes.device)
        check(self._lib.mg_query_nnz_bound(self._h, _dptr(boxes), n, _dptr(out), _stream_ptr(stream)))
        return out

    def workspace_bytes(self, max_boxes: int) -> int:
        b = ctypes.c_uint64()
        check(self._lib.mg_workspace_bytes(self._h, int(max_boxes), ctypes.byref(b)))
        return int(b.value)

    def workspace(self, max_boxes: int, stream=None):
        """Device workspace for up to max_boxes boxes per call (allocated by torch, initialised once)."""
        torch = _torch()
        if self._ws is None or self._ws_boxes < max_boxes:
            nbytes = self.workspace_bytes(max_boxes)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:%d" % self._device)
            check(self._lib.mg_workspace_init(self._h, _dptr(self._ws), nbytes, _stream_ptr(stream)))
            self._ws_boxes = max_boxes
        return self._ws

    def query(self, boxes, out=None, variant: str = "batched", workspace=None, stream=None):
        """Box histograms: boxes int32/uint32 device tensor [n, 6] -> fp32 [n, S] fractions."""
        torch = _torch()
        if boxes.dim() != 2 or boxes.shape[1] != 6 or boxes.element_size() != 4:
            raise ValueError("boxes must be a 32-bit [n, 6] tensor")
        n = boxes.shape[0]
        S = self.info()["nseg"]
        if out is None:
            out = torch.empty((n, S), dtype=torch.float32, device=boxes.device)
        if tuple(out.shape) != (n, S) or out.dtype != torch.float32:
            raise ValueError("out must be fp32 [n, S]")
        ws = workspace if workspace is not None else self.workspace(n, stream)
        fn = {"batched": self._lib.mg_query_boxes, "plain": self._lib.mg_query_boxes_plain,
              "naive": self._lib.mg_naive_boxes, "lut": self._lib.mg_query_boxes_lut}[variant]
        check(fn(self._h, _dptr(boxes), n, _dptr(out), _dptr(ws), ws.numel(), _stream_ptr(stream)))
        return out

    def query_noalloc(self, boxes, out=None, stream=None):
        """mg_query_boxes_noalloc: the batched query on the library's static device scratch (no
        workspace, no allocation inside the call). out: fp32 [n, S], allocated here if None."""
        torch = _torch()
        if boxes.dim() != 2 or boxes.shape[1] != 6 or boxes.element_size() != 4:
            raise ValueError("boxes must be a 32-bit [n, 6] tensor")
        n = boxes.shape[0]
        S = self.info()["nseg"]
        if out is None:
            out = torch.empty((n, S), dtype=torch.float32, device=boxes.device)
        if tuple(out.shape) != (n, S) or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous fp32 [n, S] tensor")
        check(self._lib.mg_query_boxes_noalloc(self._h, _dptr(boxes), n, _dptr(out), _stream_ptr(stream)))
        return out

    def query_err(self, boxes, out=None, err=None, workspace=None, stream=None):
        """Quantized graphs: (fractions fp32 [n, S], uncertainties fp32 [n, S]) from the lookup table."""
        torch = _torch()
        n = boxes.shape[0]
        S = self.info()["nseg"]
        if out is None:
            out = torch.empty((n, S), dtype=torch.float32, device=boxes.device)
        if err is None:
            err = torch.empty((n, S), dtype=torch.float32, device=boxes.device)
        ws = workspace if workspace is not None else self.workspace(n, stream)
        check(self._lib.mg_query_boxes_err(self._h, _dptr(boxes), n, _dptr(out), _dptr(err), _dptr(ws), ws.numel(),
                                           _stream_ptr(stream)))
        return out, err

    def query_stats(self, boxes, out=None, workspace=None, stream=None):
        """Batched query that also returns int32 [n, 2] (cubes, graph nodes touched) per box."""
        torch = _torch()
        n = boxes.shape[0]
        S = self.info()["nseg"]
        if out is None:
            out = torch.empty((n, S), dtype=torch.float32, device=boxes.device)
        stats = torch.zeros((n, 2), dtype=torch.int32, device=boxes.device)
        ws = workspace if workspace is not None else self.workspace(n, stream)
        check(self._lib.mg_query_boxes_stats(self._h, _dptr(boxes), n, _dptr(out), _dptr(stats), _dptr(ws),
                                             ws.numel(), _stream_ptr(stream)))
        return out, stats

    def query_sparse(self, boxes, capacity: int, workspace=None, stream=None, bufs=None):
        """Sparse histograms: (index int32 [n, 2], seg int32 [capacity], val fp32 [capacity], total int32 [1]).

        Box q's entries are seg/val[index[q,0] : index[q,0] + index[q,1]]; if total > capacity the
        call must be repeated with more room. bufs: those four tensors, preallocated (reused)."""
        torch = _torch()
        n = boxes.shape[0]
        dev = boxes.device
        if bufs is None:
            index = torch.zeros((n, 2), dtype=torch.int32, device=dev)
            seg = torch.zeros(max(capacity, 1), dtype=torch.int32, device=dev)
            val = torch.zeros(max(capacity, 1), dtype=torch.float32, device=dev)
            total = torch.zeros(1, dtype=torch.int32, device=dev)
        else:
            index, seg, val, total = bufs
            if (tuple(index.shape) != (n, 2) or seg.numel() < capacity or val.numel() < capacity
                    or total.numel() < 1):
                raise ValueError("sparse output buffers too small")
        ws = workspace if workspace is not None else self.workspace(n, stream)
        check(self._lib.mg_query_boxes_sparse(self._h, _dptr(boxes), n, _dptr(index), _dptr(seg), _dptr(val),
                                              int(capacity), _dptr(total), _dptr(ws), ws.numel(),
                                              _stream_ptr(stream)))
        return index, seg, val, total

    def footprint(self, boxes, cubes_cap: int = 0, stream=None):
        """(level counts [n, L], cubes [m, 6] or None): the GPU decomposition of each box."""
        torch = _torch()
        n = boxes.shape[0]
        L = self.info()["n_levels"]
        counts = torch.zeros((n, L), dtype=torch.int32, device=boxes.device)
        cubes = count = None
        if cubes_cap:
            cubes = torch.zeros((cubes_cap, 6), dtype=torch.int32, device=boxes.device)
            count = torch.zeros(1, dtype=torch.int32, device=boxes.device)
        check(self._lib.mg_footprint(self._h, _dptr(boxes), n, _dptr(counts),
                                     _dptr(cubes) if cubes is not None else None, int(cubes_cap),
                                     _dptr(count) if count is not None else None, _stream_ptr(stream)))
        if cubes is not None:
            m = int(count.item())
            if m > cubes_cap:
                raise RuntimeError("cube capacity %d too small (%d cubes)" % (cubes_cap, m))
            cubes = cubes[:m]
        return counts, cubes

    def propagate_tf(self, tf, out=None, stream=None):
        """RGBA8 device tensor [T, S, 4] -> fp32 [T, n_nodes, 4] node colours."""
        torch = _torch()
        T = tf.shape[0]
        inf = self.info()
        if tuple(tf.shape) != (T, inf["nseg"], 4) or tf.dtype != torch.uint8:
            raise ValueError("tf must be uint8 [T, S, 4]")
        if out is None:
            out = torch.empty((T, inf["n_nodes"], 4), dtype=torch.float32, device=tf.device)
        check(self._lib.mg_propagate_tf(self._h, _dptr(tf), T, _dptr(out), _stream_ptr(stream)))
        return out

    def palette_fetch(self, palette, level: int, xyz, out=None, stream=None):
        """Palette [T, n_nodes, 4] fp32 (from propagate_tf) at voxels xyz (uint32 [n, 3], level coords)
        -> fp32 [T, n, 4]; voxels outside the level give zeros."""
        torch = _torch()
        T = palette.shape[0]
        inf = self.info()
        if tuple(palette.shape) != (T, inf["n_nodes"], 4) or palette.dtype != torch.float32:
            raise ValueError("palette must be fp32 [T, n_nodes, 4]")
        if xyz.dim() != 2 or xyz.shape[1] != 3 or xyz.element_size() != 4:
            raise ValueError("xyz must be a 32-bit [n, 3] tensor")
        n = xyz.shape[0]
        if out is None:
            out = torch.empty((T, n, 4), dtype=torch.float32, device=palette.device)
        check(self._lib.mg_palette_fetch(self._h, _dptr(palette), T, level, _dptr(xyz), n, _dptr(out),
                                         _stream_ptr(stream)))
        return out

    def box_colour(self, palette, boxes, pal_of_box, out=None, stream=None):
        """Mean colour fp32 [n, 4] of each box under palette[pal_of_box[q]] (0xFFFFFFFF: none, zeros);
        palette fp32 [T, n_nodes, 4] from propagate_tf, boxes 32-bit [n, 6], pal_of_box 32-bit [n]."""
        torch = _torch()
        T = palette.shape[0]
        inf = self.info()
        if tuple(palette.shape) != (T, inf["n_nodes"], 4) or palette.dtype != torch.float32:
            raise ValueError("palette must be fp32 [T, n_nodes, 4]")
        n = boxes.shape[0]
        if boxes.dim() != 2 or boxes.shape[1] != 6 or boxes.element_size() != 4:
            raise ValueError("boxes must be a 32-bit [n, 6] tensor")
        if pal_of_box.shape != (n,) or pal_of_box.element_size() != 4:
            raise ValueError("pal_of_box must be a 32-bit [n] tensor")
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=palette.device)
        check(self._lib.mg_box_colour(self._h, _dptr(palette), T, _dptr(boxes), n, _dptr(pal_of_box), _dptr(out),
                                      _stream_ptr(stream)))
        return out

    def lut_build(self, threads: int = 0) -> int:
        """Build (and upload, if on a device) the mixture lookup table; returns its entry count."""
        nnz = ctypes.c_uint64(0)
        check(self._lib.mg_lut_build(self._h, threads, ctypes.byref(nnz)))
        return int(nnz.value)

    def export_lut(self, with_err: bool = False):
        """(ptr uint64 [n_nodes + 1], seg uint32 [nnz], val float32 [nnz][, err float32 [nnz]]) of the
        mixture lookup table; err is the propagated uncertainty of each fraction."""
        N = self.info()["n_nodes"]
        ptr = np.zeros(N + 1, dtype=np.uint64)
        check(self._lib.mg_export_lut(self._h, ptr.ctypes.data, None, None, None))
        nnz = int(ptr[-1])
        seg = np.zeros(nnz, dtype=np.uint32)
        val = np.zeros(nnz, dtype=np.float32)
        err = np.zeros(nnz, dtype=np.float32)
        check(self._lib.mg_export_lut(self._h, ptr.ctypes.data, seg.ctypes.data, val.ctypes.data,
                                      err.ctypes.data if with_err else None))
        return (ptr, seg, val, err) if with_err else (ptr, seg, val)

    def quantize(self, bits: int, threads: int = 0) -> "Graph":
        """Lossy copy with scalar-quantized weights (2^bits bins) and merged nodes."""
        h = ctypes.c_void_p()
        check(self._lib.mg_quantize(self._h, bits, threads, ctypes.byref(h)))
        return Graph(h)

    def export_codebook(self, with_code: bool = False):
        """(codeword fp32 [2^bits], sigma fp32 [2^bits], node_sigma fp32 [n_nodes][, node_code u32 [n_nodes]])
        of a quantized graph."""
        inf = self.info()
        B = 1 << inf["quant_bits"] if inf["quant_bits"] else 0
        cw = np.zeros(max(B, 1), dtype=np.float32)
        sg = np.zeros(max(B, 1), dtype=np.float32)
        ns = np.zeros(inf["n_nodes"], dtype=np.float32)
        nc = np.zeros(inf["n_nodes"], dtype=np.uint32)
        check(self._lib.mg_export_codebook(self._h, cw.ctypes.data, sg.ctypes.data, ns.ctypes.data, nc.ctypes.data))
        return (cw, sg, ns, nc) if with_code else (cw, sg, ns)

    def launch_config(self) -> dict:
        c = LaunchCfg()
        check(self._lib.mg_get_launch(self._h, ctypes.byref(c)))
        return {"unroll_big": c.unroll_big, "unroll_small": c.unroll_small, "unroll_naive": c.unroll_naive,
                "tf_block": c.tf_block, "table_big": c.table_big, "table_small": c.table_small,
                "table_retry": c.table_retry, "block_small": c.block_small, "block_big": c.block_big,
                "chunk_small": c.chunk_small, "tf_planes": c.tf_planes, "tf_schedule": c.tf_schedule,
                "run_min_row": c.run_min_row}

    def set_launch_config(self, **kw) -> None:
        cur = self.launch_config()
        cur.update(kw)
        c = LaunchCfg(**cur)
        check(self._lib.mg_set_launch(self._h, ctypes.byref(c)))

    def autotune(self, boxes, out=None, reps: int = 3, workspace=None, stream=None) -> dict:
        """mg_autotune on these boxes: keeps and returns the fastest launch configuration."""
        torch = _torch()
        n = boxes.shape[0]
        if out is None:
            out = torch.empty((n, self.info()["nseg"]), dtype=torch.float32, device=boxes.device)
        ws = workspace if workspace is not None else self.workspace(n, stream)
        c = LaunchCfg()
        check(self._lib.mg_autotune(self._h, _dptr(boxes), n, _dptr(out), _dptr(ws), ws.numel(), int(reps),
                                    _stream_ptr(stream), ctypes.byref(c)))
        return self.launch_config()

    def timing(self, enable: bool) -> None:
        check(self._lib.mg_timing_enable(self._h, 1 if enable else 0))

    def timing_read(self):
        ms = ctypes.c_double()
        k = ctypes.c_uint32()
        check(self._lib.mg_timing_read(self._h, ctypes.byref(ms), ctypes.byref(k)))
        return float(ms.value), int(k.value)
