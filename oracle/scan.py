"""O1: brute-force box histograms over the level-0 segment volume (ground truth).

ORACLE (test infrastructure only). Definition followed: the histogram of a
sub-volume counts, for every segment ID, the level-0 voxels of the box that
carry it (Sec. "Fast Sub-Volume Queries"); normalised, it is the box's mixture
(Sec. 3, Notation: a convex, finitely supported vector). Box readings: the
extent is a voxel count, the range is half-open ``[x0, x0+dx)``, and the box
is clipped to the volume, an origin at or past the volume giving an empty box
(the clipping step of the appendix algorithm).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "o1_scan.c")
_LIB = os.path.join(_HERE, "libo1.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile o1_scan.c (gcc -O3 -fopenmp) into oracle/libo1.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i64 = ctypes.c_void_p, ctypes.c_int64
        lib.o1_box_counts.argtypes = [vp, i64, i64, i64, i64, vp, i64, vp, vp, ctypes.c_int]
        lib.o1_box_counts.restype = ctypes.c_int
        lib.o1_max_threads.restype = ctypes.c_int
        lib.o1_compact.argtypes = [vp, i64, ctypes.c_uint32, vp, vp, ctypes.c_int]
        lib.o1_compact.restype = i64
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().o1_max_threads())


def compact(vol: np.ndarray, threads: int = 0):
    """Segment IDs in increasing order and the volume as indices into them (uint32).

    Volumes whose largest ID is below 2^28 go through a table of all IDs up to the largest (C,
    linear time); others through numpy.unique."""
    vol = np.asarray(vol)
    flat = np.ascontiguousarray(vol.ravel(), dtype=np.uint32) if vol.dtype != np.uint32 else \
        np.ascontiguousarray(vol).ravel()
    mx = int(flat.max()) if flat.size else 0
    if mx >= (1 << 28):
        ids, inv = np.unique(flat, return_inverse=True)
        return ids.astype(np.uint64), inv.astype(np.uint32).reshape(vol.shape)
    lut = np.zeros(mx + 1, dtype=np.uint32)
    out = np.empty(flat.size, dtype=np.uint32)
    k = _load().o1_compact(flat.ctypes.data, flat.size, mx, lut.ctypes.data, out.ctypes.data, int(threads))
    if k < 0:
        raise RuntimeError("o1_compact failed")
    ids = np.nonzero(lut)[0].astype(np.uint64)
    assert len(ids) == k
    return ids, out.reshape(vol.shape)


def clipped(box, dims):
    """Half-open clipped ranges ((x0, x1), (y0, y1), (z0, z1)); empty ranges have x1 <= x0."""
    out = []
    for a in range(3):
        lo = int(box[a])
        hi = min(lo + int(box[3 + a]), int(dims[a]))
        out.append((lo, max(hi, lo)))
    return tuple(out)


def box_counts(vol_c: np.ndarray, nseg: int, boxes: np.ndarray, threads: int = 0, probs: bool = True):
    """uint64 counts [n, nseg] (and fp64 fractions) of compacted volume ``vol_c`` (shape (nz, ny, nx))."""
    vol_c = np.ascontiguousarray(vol_c, dtype=np.uint32)
    boxes = np.ascontiguousarray(boxes, dtype=np.uint32).reshape(-1, 6)
    nz, ny, nx = vol_c.shape
    n = len(boxes)
    counts = np.zeros((n, nseg), dtype=np.uint64)
    pr = np.zeros((n, nseg), dtype=np.float64) if probs else None
    rc = _load().o1_box_counts(vol_c.ctypes.data, nx, ny, nz, int(nseg), boxes.ctypes.data, n,
                               counts.ctypes.data, pr.ctypes.data if probs else None, int(threads))
    if rc != 0:
        raise RuntimeError("o1_box_counts failed (%d)" % rc)
    return (counts, pr) if probs else counts


def box_histogram(vol: np.ndarray, boxes: np.ndarray, threads: int = 0):
    """Segment IDs, uint64 counts [n, S] and fp64 fractions [n, S] for an uncompacted ID volume."""
    ids, vol_c = compact(vol)
    counts, pr = box_counts(vol_c, len(ids), boxes, threads)
    return ids, counts, pr


def box_counts_numpy(vol_c: np.ndarray, nseg: int, box) -> np.ndarray:
    """One box by slicing and numpy.bincount (the library routine the C scan must agree with)."""
    nz, ny, nx = vol_c.shape
    (x0, x1), (y0, y1), (z0, z1) = clipped(box, (nx, ny, nz))
    sl = vol_c[z0:z1, y0:y1, x0:x1]
    return np.bincount(sl.ravel().astype(np.int64), minlength=nseg).astype(np.uint64)
