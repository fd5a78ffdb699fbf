"""Voxel downsampling of the accumulated LiDAR cloud (Sec. III-C: one point per voxel,
coarse-to-fine voxel sizes) -- test infrastructure only.

Voxel of a point: floor((x - lo) / voxel) per axis in float64; every coordinate must
lie in [0, 2^21).  One point is kept per occupied voxel, the one with the lowest
index.  The paper fixes no order for the kept points; they are listed in Morton
(Z-curve) order of their voxels -- bit b of the x, y and z coordinates becomes bit
3b, 3b + 1 and 3b + 2 of the code -- so that points close in space stay close in
memory.
"""
from __future__ import annotations

import numpy as np

__all__ = ["voxel_keys", "morton_code", "downsample", "VOXEL_BITS"]

VOXEL_BITS = 21


def voxel_keys(pts, lo, voxel):
    """Integer voxel coordinates [n,3] (int64) of points pts [3,n]."""
    p = np.asarray(pts, np.float64)
    return np.floor((p.T - np.asarray(lo, np.float64)) / float(voxel)).astype(np.int64)


def morton_code(k):
    """Z-curve code of voxel coordinates k [n,3]: bit b of axis d goes to bit 3b + d."""
    k = np.asarray(k, np.int64)
    if k.size and (k.min() < 0 or k.max() >= (1 << VOXEL_BITS)):
        raise ValueError("voxel coordinates outside [0, 2^21)")
    code = np.zeros(k.shape[0], np.uint64)
    for b in range(VOXEL_BITS):
        for d in range(3):
            bit = (k[:, d] >> b) & 1
            code |= bit.astype(np.uint64) << np.uint64(3 * b + d)
    return code


def downsample(pts, lo, voxel):
    """Indices of the kept points (lowest index per voxel), in Morton order of the voxels."""
    code = morton_code(voxel_keys(pts, lo, voxel))
    _, first = np.unique(code, return_index=True)   # sorted by code; first = lowest index
    return first.astype(np.int64)
