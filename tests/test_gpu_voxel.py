"""GPU parity of the voxel downsampling (one point per voxel, the lowest index, in
Z-curve order of the voxels; Sec. III-C coarse-to-fine stages) against the oracle: the
kept indices must be identical, bit for bit."""
import numpy as np
import pytest
import torch

import oracle
from synth import scenes
from paper_2403_11577_amd import binding as B

from gpu_util import say

pytestmark = pytest.mark.gpu


def _gpu_downsample(pts, lo, voxel, ws=None):
    n = pts.shape[1]
    d = torch.as_tensor(np.ascontiguousarray(pts, np.float32), device="cuda")
    need = B.splat_voxel_workspace_size(n)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device="cuda")
    keep = torch.full((max(n, 1),), -7, dtype=torch.int32, device="cuda")
    n_keep = torch.full((1,), 123456, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    B.splat_voxel_downsample(d, lo, voxel, ws, keep, n_keep, status)
    torch.cuda.synchronize()
    m = int(n_keep.item())
    return keep[:m].cpu().numpy().astype(np.int64), int(status.item()), keep, ws


def _cloud(seed, n):
    rng = np.random.default_rng(seed)
    pts = rng.uniform([-3, -2, 0], [4, 5, 2], size=(n, 3)).astype(np.float32)
    if n >= 310:
        pts[100:200] = pts[100]                       # duplicates
        pts[300:310, 0] = np.float32(-3.0 + 0.25 * 5)  # on a voxel face
    return pts.T.copy()


@pytest.mark.parametrize("n, voxel", [(1, 0.1), (3000, 0.25), (3000, 10.0), (200_000, 0.05), (1_000_003, 0.02)])
def test_voxel_downsample_matches_the_oracle(n, voxel):
    say(f"voxel n={n} v={voxel}")
    pts, lo = _cloud(n, n), np.array([-3.0, -2.0, 0.0])
    got, status, keep, _ = _gpu_downsample(pts, lo, voxel)
    want = oracle.downsample(pts, lo, voxel)
    assert status == 0
    np.testing.assert_array_equal(got, want)
    assert np.all(keep[len(got):].cpu().numpy() == -7)  # nothing written past n_keep


def test_voxel_downsample_accumulated_drive_cloud_coarse_to_fine():
    """The paper's input: LiDAR scans accumulated over a drive (4.5 M returns),
    downsampled at the three stages of the schedule, workspace reused."""
    pts = scenes.drive_scans(seed=0)
    lo = np.floor(pts.min(axis=1).astype(np.float64)) - 0.5
    ws = None
    for voxel in (0.10, 0.05, 0.02):
        say(f"drive cloud n={pts.shape[1]} v={voxel}")
        got, status, _, ws = _gpu_downsample(pts, lo, voxel, ws)
        want = oracle.downsample(pts, lo, voxel)
        assert status == 0
        say(f"  kept {len(got)} of {pts.shape[1]}")
        np.testing.assert_array_equal(got, want)


def test_voxel_downsample_of_nothing_and_of_the_result():
    pts, lo = _cloud(5, 5000), np.array([-3.0, -2.0, 0.0])
    got, status, _, _ = _gpu_downsample(pts[:, :0], lo, 0.1)
    assert len(got) == 0 and status == 0
    keep, _, _, _ = _gpu_downsample(pts, lo, 0.3)
    again, _, _, _ = _gpu_downsample(pts[:, keep], lo, 0.3)
    np.testing.assert_array_equal(again, np.arange(len(keep)))  # already one point per voxel, in voxel order


def test_voxel_downsample_flags_points_outside_the_grid():
    pts, lo = _cloud(6, 4000), np.array([-3.0, -2.0, 0.0])
    pts[1, 17] = -2.5                    # below lo on y
    pts[0, 18] = np.nan
    got, status, _, _ = _gpu_downsample(pts, lo, 0.2)
    assert status & 16                   # SPLAT_ST_RANGE
    # every other point is still placed by the definition
    ok = np.ones(pts.shape[1], bool)
    ok[[17, 18]] = False
    k = oracle.voxel_keys(pts[:, ok], lo, 0.2)
    assert len(got) >= len({tuple(r) for r in k})
