"""Normalized histogram mipmap, written out from the level-0 volume.

ORACLE (test infrastructure only). Follows Eq. (mip), Sec. "Normalized
Histogram Mipmap": level 0 holds the unit vector of each voxel's segment;
level l averages the (at most 8) level-(l-1) children; resolutions are rounded
up per level until a single voxel remains.

Readings:
- Levels: each axis halves with rounding up, ceil(d/2), until every axis is 1,
  so there are ceil(log2(max dim)) + 1 levels.
- Border weights: "N is the number of voxels in the support" is read as the
  number of level-0 voxels under the mip voxel (``mode="voxels"``, the
  default): every mip voxel then holds the exact normalized histogram of its
  level-0 support, i.e. integer counts divided by their sum. The literal
  alternative, the number of children averaged (``mode="children"``), is
  also available; the two differ only at non-power-of-two borders.

Computed by definition: counts of a mip voxel are counted over its clipped
level-0 support, not derived from the level below.
"""
from __future__ import annotations

import numpy as np


def level_dims(dims):
    """[(nx, ny, nz) of level 0, level 1, ...] down to (1, 1, 1)."""
    d = tuple(int(v) for v in dims)
    out = [d]
    while any(v > 1 for v in d):
        d = tuple((v + 1) // 2 for v in d)
        out.append(d)
    return out


def total_voxels(dims) -> int:
    return sum(int(np.prod(d, dtype=np.int64)) for d in level_dims(dims))


def support(dims, level: int, v):
    """Clipped half-open level-0 ranges ((x0,x1),(y0,y1),(z0,z1)) under mip voxel v at ``level``."""
    s = 1 << level
    return tuple((int(v[a]) * s, min((int(v[a]) + 1) * s, int(dims[a]))) for a in range(3))


def counts_level(vol_c: np.ndarray, nseg: int, level: int) -> np.ndarray:
    """int64 [nz_l, ny_l, nx_l, nseg]: per mip voxel, level-0 voxel count of each segment in its support."""
    nz, ny, nx = vol_c.shape
    s = 1 << level
    lx, ly, lz = level_dims((nx, ny, nz))[level]
    out = np.zeros((lz, ly, lx, nseg), dtype=np.int64)
    z_idx = (np.arange(nz) // s)[:, None, None]
    y_idx = (np.arange(ny) // s)[None, :, None]
    x_idx = (np.arange(nx) // s)[None, None, :]
    zz, yy, xx = np.broadcast_arrays(z_idx, y_idx, x_idx)
    np.add.at(out, (zz.ravel(), yy.ravel(), xx.ravel(), vol_c.ravel().astype(np.int64)), 1)
    return out


def mixtures_level(vol_c: np.ndarray, nseg: int, level: int, mode: str = "voxels") -> np.ndarray:
    """fp64 [nz_l, ny_l, nx_l, nseg]: the normalized histogram H(., level)."""
    if mode == "voxels":
        c = counts_level(vol_c, nseg, level).astype(np.float64)
        return c / c.sum(axis=-1, keepdims=True)
    if mode == "children":
        h = np.zeros(vol_c.shape + (nseg,), dtype=np.float64)
        zi, yi, xi = np.indices(vol_c.shape)
        h[zi, yi, xi, vol_c.astype(np.int64)] = 1.0
        for _ in range(level):
            nz, ny, nx = h.shape[:3]
            lz, ly, lx = (nz + 1) // 2, (ny + 1) // 2, (nx + 1) // 2
            acc = np.zeros((lz, ly, lx, nseg), dtype=np.float64)
            cnt = np.zeros((lz, ly, lx, 1), dtype=np.float64)
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        sub = h[dz::2, dy::2, dx::2]
                        acc[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += sub
                        cnt[:sub.shape[0], :sub.shape[1], :sub.shape[2]] += 1.0
            h = acc / cnt
        return h
    raise ValueError(mode)
