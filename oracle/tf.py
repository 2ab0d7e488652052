"""Transfer-function colours of mip voxels, straight from the volume.

ORACLE (test infrastructure only). A node's colour is the scalar product of
its mixture with the per-segment colours (Sec. 3, Notation: a mixture times a
data vector is a convex combination of its entries; Sec. "Reconstruction":
colours assigned to the sources are propagated to every node; Sec.
"Rendering": the node ID of a mip voxel indexes that colour table). So the
colour of a mip voxel is the mixture-weighted mean of its segments' colours,
computed here from the mipmap definition (``mipmap.mixtures_level``).

Colours: RGBA8 bytes read as value/255 in fp64.
"""
from __future__ import annotations

import numpy as np

from . import mipmap


def rgba_to_float(tf_u8: np.ndarray) -> np.ndarray:
    return np.asarray(tf_u8, dtype=np.float64) / 255.0


def level_colours(vol_c: np.ndarray, nseg: int, tf_u8: np.ndarray, level: int, mode: str = "voxels") -> np.ndarray:
    """fp64 [nz_l, ny_l, nx_l, 4]: mean colour of each mip voxel of ``level`` for one TF [nseg, 4]."""
    h = mipmap.mixtures_level(vol_c, nseg, level, mode)
    return h @ rgba_to_float(tf_u8)


def voxel_colour(vol_c: np.ndarray, tf_u8: np.ndarray, level: int, v) -> np.ndarray:
    """Mean colour over the level-0 support of one mip voxel (voxel-count weights), fp64 [4]."""
    nz, ny, nx = vol_c.shape
    (x0, x1), (y0, y1), (z0, z1) = mipmap.support((nx, ny, nz), level, v)
    seg = vol_c[z0:z1, y0:y1, x0:x1].ravel().astype(np.int64)
    return rgba_to_float(tf_u8)[seg].mean(axis=0)
