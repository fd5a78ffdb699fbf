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


def _z_less(a, b):
    """a before b on the Z-curve: compare on the axis whose coordinates differ in the
    highest bit (ties between axes go to the later axis), then by that axis."""
    best, axis = -1, 0
    for d in range(3):
        x = a[d] ^ b[d]
        if x and x.bit_length() - 1 >= best:
            best, axis = x.bit_length() - 1, d
    return a[axis] < b[axis]


def test_kept_points_come_in_morton_order_of_their_voxels():
    pts, lo = _cloud(1), np.array([-3.0, -2.0, 0.0])
    keep = oracle.downsample(pts, lo, 0.5)
    k = oracle.voxel_keys(pts, lo, 0.5)[keep]
    for i in range(len(keep) - 1):
        assert _z_less(tuple(int(v) for v in k[i]), tuple(int(v) for v in k[i + 1]))


def test_morton_code_of_small_coordinates():
    # bit b of x, y, z -> bits 3b, 3b+1, 3b+2
    k = np.array([[1, 0, 0], [0, 1, 0], [0, 0, 1], [3, 0, 0], [7, 7, 7], [0, 0, (1 << 21) - 1]])
    want = [1, 2, 4, 0b1001, (1 << 9) - 1, sum(4 << (3 * b) for b in range(21))]
    assert oracle.morton_code(k).tolist() == want
    with pytest.raises(ValueError):
        oracle.morton_code(np.array([[0, -1, 0]]))
    with pytest.raises(ValueError):
        oracle.morton_code(np.array([[1 << 21, 0, 0]]))


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
    assert len(oracle.downsample(pts, lo, 1e-5)) == distinct


def test_voxel_keys_follow_the_floor_definition_at_boundaries():
    pts = np.array([[0.0, 0.25, 0.2499999999, -1e-12], [0, 0, 0, 0], [0, 0, 0, 0]])
    k = oracle.voxel_keys(pts, np.zeros(3), 0.25)
    assert k[:, 0].tolist() == [0, 1, 0, -1]
