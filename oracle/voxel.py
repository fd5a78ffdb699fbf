"""Voxel downsampling of the accumulated LiDAR cloud (Sec. III-C: one point per voxel,
coarse-to-fine voxel sizes) -- test infrastructure only.

Voxel of a point: floor((x - lo) / voxel) per axis in float64.  One point is kept per
occupied voxel, the one with the lowest index; the kept indices are listed in voxel
order (z major, then y, then x).
"""
from __future__ import annotations

import numpy as np

__all__ = ["voxel_keys", "downsample"]


def voxel_keys(pts, lo, voxel):
    """Integer voxel coordinates [n,3] (int64) of points pts [3,n]."""
    p = np.asarray(pts, np.float64)
    return np.floor((p.T - np.asarray(lo, np.float64)) / float(voxel)).astype(np.int64)


def downsample(pts, lo, voxel):
    """Indices of the kept points (lowest index per voxel), in (z, y, x) voxel order."""
    k = voxel_keys(pts, lo, voxel)
    _, first = np.unique(k[:, ::-1], axis=0, return_index=True)   # rows sorted by (z, y, x)
    return first.astype(np.int64)
