"""Pins of the voxel downsampling oracle (one point per voxel, Sec. III-C)."""
import numpy as np
import pytest

import oracle


def _cloud(seed, n=3000):
    rng = np.random.default_rng(seed)
    pts = rng.uniform([-3, -2, 0], [4, 5, 2], size=(n, 3))
    pts[100:200] = pts[100]  # duplicates
    return pts.T.copy()


def test_one_point_per_occupied_voxel_and_the_lowest_index():
    pts, lo, v = _cloud(0), np.array([-3.0, -2.0, 0.0]), 0.25
    keep = oracle.downsample(pts, lo, v)
    k = oracle.voxel_keys(pts, lo, v)
    occupied = {tuple(r) for r in k}
    assert len(keep) == len(occupied)
    assert len({tuple(k[i]) for i in keep}) == len(keep)
    # brute force: the smallest index of every voxel
    best = {}
    for i, r in enumerate(map(tuple, k)):
        best.setdefault(r, i)
    assert sorted(keep.tolist()) == sorted(best.values())


def test_kept_points_come_in_z_y_x_voxel_order():
    pts, lo = _cloud(1), np.array([-3.0, -2.0, 0.0])
    keep = oracle.downsample(pts, lo, 0.5)
    k = oracle.voxel_keys(pts, lo, 0.5)[keep]
    packed = (k[:, 2] << 42) | (k[:, 1] << 21) | k[:, 0]
    assert np.all(np.diff(packed) > 0)


def test_downsampling_the_result_again_keeps_everything():
    pts, lo, v = _cloud(2), np.array([-3.0, -2.0, 0.0]), 0.3
    keep = oracle.downsample(pts, lo, v)
    sub = pts[:, keep]
    again = oracle.downsample(sub, lo, v)
    assert sorted(again.tolist()) == list(range(sub.shape[1]))


@pytest.mark.parametrize("v", [0.1, 0.05, 0.02])
def test_finer_voxels_keep_more_points_and_a_fine_enough_grid_keeps_all(v):
    pts, lo = _cloud(3), np.array([-3.0, -2.0, 0.0])
    n_coarse = len(oracle.downsample(pts, lo, 2 * v))
    n_fine = len(oracle.downsample(pts, lo, v))
    assert n_fine >= n_coarse
    distinct = len({tuple(c) for c in pts.T})
    assert len(oracle.downsample(pts, lo, 1e-9)) == distinct


def test_voxel_keys_follow_the_floor_definition_at_boundaries():
    pts = np.array([[0.0, 0.25, 0.2499999999, -1e-12], [0, 0, 0, 0], [0, 0, 0, 0]])
    k = oracle.voxel_keys(pts, np.zeros(3), 0.25)
    assert k[:, 0].tolist() == [0, 1, 0, -1]
