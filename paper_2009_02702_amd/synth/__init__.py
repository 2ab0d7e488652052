"""Seeded synthetic inputs: segmentation volumes, box queries, transfer functions.

This module is input generation only. It holds none of the Mixture Graph
method's arithmetic (no mipmap, footprint, factorization or push), so both
the HIP path and the CPU oracle may draw their inputs from it.

Random draws come from NumPy's PCG64 seeded with ``(20090270 + config, stream)``
through a ``SeedSequence``; the rasterisation of those draws into a label
volume is done by ``gen.c`` (deterministic, any thread count).

The five workloads stand in for the paper's three segmentation datasets
(Hippocampus 1178x1125x789 / 353 segments, Neocortex 2048^2x300 / 1,182,
Polymer 614x961x600 / 15,917; Sec. Results, Table "resultsFactorization"),
which are not available: synthetic volumes with the same shapes and segment
counts, Voronoi cells for the two neuro volumes and random capsules for the
fibre-reinforced polymer.

Volumes are uint32 (config 1 is uint16 by recipe), x fastest:
``vol[z, y, x]`` in NumPy order, i.e. flat index ``x + nx*(y + ny*z)``.
Boxes are uint32 ``[n, 6]`` rows ``(x0, y0, z0, dx, dy, dz)``: the half-open
voxel range ``[x0, x0+dx) x [y0, y0+dy) x [z0, z0+dz)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

SEED_BASE = 20090270


def build(force: bool = True) -> str:
    """Compile gen.c into libsynth.so (gcc -O3 -fopenmp)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            raise RuntimeError("libsynth.so is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(_LIB)
        i64, u32, dp, vp = ctypes.c_int64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p
        lib.synth_voronoi.argtypes = [vp, i64, i64, i64, dp, i64, ctypes.c_double, u32, i64, i64, i64]
        lib.synth_voronoi_brute.argtypes = [vp, i64, i64, i64, dp, i64, ctypes.c_double, u32]
        lib.synth_cell_sums.argtypes = [vp, i64, i64, i64, u32, i64, dp, vp]
        lib.synth_cylinders.argtypes = [vp, i64, i64, i64, dp, i64]
        lib.synth_cylinders_brute.argtypes = [vp, i64, i64, i64, dp, i64]
        for f in (lib.synth_voronoi, lib.synth_voronoi_brute, lib.synth_cell_sums,
                  lib.synth_cylinders, lib.synth_cylinders_brute):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def rng(config: int, stream: int) -> np.random.Generator:
    """PCG64 stream ``stream`` of workload ``config`` (0: volume, 1: boxes, 2: TFs, 3: arrivals)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([SEED_BASE + config, stream])))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def voronoi(dims, seeds: np.ndarray, zscale: float = 1.0, base: int = 1, brute: bool = False) -> np.ndarray:
    """Label volume: base + index of the nearest seed (ties to the lower index)."""
    nx, ny, nz = (int(d) for d in dims)
    seeds = np.ascontiguousarray(seeds, dtype=np.float64)
    out = np.empty((nz, ny, nx), dtype=np.uint32)
    lib = _load()
    if brute:
        rc = lib.synth_voronoi_brute(_ptr(out), nx, ny, nz, seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     len(seeds), float(zscale), base)
    else:
        bz = max(1, int(round(16 / max(zscale, 1e-9))))
        rc = lib.synth_voronoi(_ptr(out), nx, ny, nz, seeds.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                               len(seeds), float(zscale), base, 16, 16, min(bz, 16))
    if rc != 0:
        raise RuntimeError("synth_voronoi failed (%d)" % rc)
    return out


def lloyd_step(vol: np.ndarray, seeds: np.ndarray, base: int = 1) -> np.ndarray:
    """One Lloyd step: every seed moves to the centroid of its cell's voxel centres; empty cells keep theirs."""
    nz, ny, nx = vol.shape
    k = len(seeds)
    sums = np.zeros(3 * k, dtype=np.float64)
    counts = np.zeros(k, dtype=np.int64)
    rc = _load().synth_cell_sums(_ptr(vol), nx, ny, nz, base, k,
                                 sums.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), _ptr(counts))
    if rc != 0:
        raise RuntimeError("synth_cell_sums failed (%d)" % rc)
    out = np.array(seeds, dtype=np.float64, copy=True)
    nz_ = counts > 0
    out[nz_] = sums.reshape(k, 3)[nz_] / counts[nz_, None]
    return out


def cylinders(dims, params: np.ndarray, brute: bool = False) -> np.ndarray:
    """Capsules painted in order over background 0; capsule i gets label i+1."""
    nx, ny, nz = (int(d) for d in dims)
    params = np.ascontiguousarray(params, dtype=np.float64)
    assert params.ndim == 2 and params.shape[1] == 8
    out = np.zeros((nz, ny, nx), dtype=np.uint32)
    lib = _load()
    fn = lib.synth_cylinders_brute if brute else lib.synth_cylinders
    rc = fn(_ptr(out), nx, ny, nz, params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(params))
    if rc != 0:
        raise RuntimeError("synth_cylinders failed (%d)" % rc)
    return out


# --------------------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------------------

@dataclass
class Workload:
    """One synthetic workload: volume recipe + query recipe, at full or reduced size."""
    config: int
    name: str
    dims: tuple
    segments: int
    n_boxes: int
    kind: str                      # "voronoi" | "cylinders"
    zscale: float = 1.0
    lloyd: bool = False
    box_mode: str = "loguniform"   # "corners" | "loguniform" | "mixed"
    tf_count: int = 0
    volume_dtype: str = "uint32"
    extra: dict = field(default_factory=dict)


FULL = {
    1: Workload(1, "voronoi64_16seg_1k", (64, 64, 64), 16, 1000, "voronoi",
                box_mode="corners", volume_dtype="uint16"),
    2: Workload(2, "voronoi512_353seg_100k", (512, 512, 512), 353, 100_000, "voronoi", lloyd=True),
    3: Workload(3, "aniso2048x2048x300_1182seg_50k_tf8", (2048, 2048, 300), 1182, 50_000, "voronoi",
                zscale=7.0, tf_count=8),
    4: Workload(4, "cylinders614x961x600_15917seg_1m", (614, 961, 600), 15917, 1_000_000, "cylinders",
                box_mode="mixed"),
    5: Workload(5, "voronoi1178x1125x789_353seg_stream", (1178, 1125, 789), 353, 200_000, "voronoi",
                tf_count=1),
}


def workload(config: int, dims: Optional[tuple] = None, segments: Optional[int] = None,
             n_boxes: Optional[int] = None) -> Workload:
    """The recipe of a workload, optionally at reduced dims / segment count / query count."""
    w = FULL[config]
    return Workload(w.config, w.name, tuple(dims) if dims else w.dims, segments or w.segments,
                    n_boxes if n_boxes is not None else w.n_boxes, w.kind, w.zscale, w.lloyd, w.box_mode,
                    w.tf_count, w.volume_dtype, dict(w.extra))


def make_volume(w: Workload) -> np.ndarray:
    """Label volume of workload ``w`` (NumPy shape (nz, ny, nx), x fastest)."""
    nx, ny, nz = w.dims
    g = rng(w.config, 0)
    if w.kind == "voronoi":
        seeds = g.random((w.segments, 3)) * np.array([nx, ny, nz], dtype=np.float64)
        vol = voronoi(w.dims, seeds, zscale=w.zscale, base=1)
        if w.lloyd:
            seeds = lloyd_step(vol, seeds, base=1)
            vol = voronoi(w.dims, seeds, zscale=w.zscale, base=1)
    elif w.kind == "cylinders":
        k = w.segments
        centre = g.random((k, 3)) * np.array([nx, ny, nz], dtype=np.float64)
        axis = g.standard_normal((k, 3))
        axis /= np.linalg.norm(axis, axis=1, keepdims=True)
        radius = g.uniform(2.0, 6.0, k)
        length = g.uniform(20.0, 300.0, k)
        half = (0.5 * length)[:, None] * axis
        params = np.zeros((k, 8), dtype=np.float64)
        params[:, 0:3] = centre - half
        params[:, 3:6] = centre + half
        params[:, 6] = radius
        vol = cylinders(w.dims, params)
    else:
        raise ValueError(w.kind)
    if w.volume_dtype == "uint16":
        assert int(vol.max()) < 65536
        vol = vol.astype(np.uint16)
    return vol


def make_boxes(w: Workload, n: Optional[int] = None) -> np.ndarray:
    """Box queries of workload ``w`` as uint32 [n, 6] rows (x0, y0, z0, dx, dy, dz)."""
    n = w.n_boxes if n is None else int(n)
    dims = np.array(w.dims, dtype=np.int64)
    g = rng(w.config, 1)
    if w.box_mode == "corners":
        # two corners per axis uniform over the voxels; lo = min, extent = |c - c'| + 1
        c0 = g.integers(0, dims, size=(n, 3))
        c1 = g.integers(0, dims, size=(n, 3))
        lo = np.minimum(c0, c1)
        ext = np.abs(c0 - c1) + 1
    else:
        # per axis: extent e = round(D^U), U ~ U[0,1), clamped to [1, D]; origin uniform in [0, D - e]
        u = g.random((n, 3))
        ext = np.clip(np.rint(np.power(dims[None, :].astype(np.float64), u)).astype(np.int64), 1, dims[None, :])
        lo = (g.random((n, 3)) * (dims[None, :] - ext + 1)).astype(np.int64)
        lo = np.minimum(lo, dims[None, :] - ext)
        if w.box_mode == "mixed" and n > 0:
            # forced share of full-volume boxes (0.1%) and single voxels (1%)
            r = g.random(n)
            full = r < 0.001
            one = (r >= 0.001) & (r < 0.011)
            lo[full] = 0
            ext[full] = dims
            ext[one] = 1
    boxes = np.concatenate([lo, ext], axis=1).astype(np.uint32)
    return np.ascontiguousarray(boxes)


def make_tfs(w: Workload, n_segments: int, t: Optional[int] = None) -> np.ndarray:
    """Random RGBA8 transfer functions, uint8 [T, S, 4] (one colour per compacted segment)."""
    t = w.tf_count if t is None else int(t)
    g = rng(w.config, 2)
    return np.ascontiguousarray(g.integers(0, 256, size=(t, n_segments, 4), dtype=np.uint8))


def poisson_arrivals(w: Workload, n: int, qps: float) -> np.ndarray:
    """Arrival times in seconds of ``n`` requests of a Poisson process at rate ``qps``."""
    g = rng(w.config, 3)
    return np.cumsum(g.exponential(1.0 / float(qps), size=int(n)))
