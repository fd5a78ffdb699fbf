"""Pins of the binning reference: tile lists cover every contributing pixel and
are in (depth32, Gaussian id) order, so images do not depend on the tile size."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (16, 32)])
def test_tile_lists_cover_contributors_in_order(tile):
    s = synth.tiny_scene(0)
    w2c = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)[0]
    intr = oracle.view_intr(s.rig, s.views)
    W, H = s.rig.W, s.rig.H
    proj = oracle.project_all(s.gauss, w2c, intr, W, H)
    off, gid, margin = oracle.tile_lists(proj, W, H, tile[0], tile[1])
    tx_n = (W + tile[0] - 1) // tile[0]
    dep = proj["depth32"][0]
    # order inside every tile: ascending depth32, then id
    for t in range(len(off) - 1):
        ids = gid[off[t]:off[t + 1]]
        key = list(zip(dep[ids], ids))
        assert key == sorted(key)
    rng = np.random.default_rng(0)
    for _ in range(60):
        x, y = int(rng.integers(W)), int(rng.integers(H))
        st = oracle.pixel_stack(s.gauss, w2c[0], intr[0], W, H, x, y)
        t = (y // tile[1]) * tx_n + x // tile[0]
        lst = list(gid[off[t]:off[t + 1]])
        pos = [lst.index(int(g)) for g in st[:, 0]]
        assert pos == sorted(pos)


def test_tile_counts_grow_with_smaller_tiles():
    s = synth.tiny_scene(0)
    w2c = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)[0]
    intr = oracle.view_intr(s.rig, s.views)
    proj = oracle.project_all(s.gauss, w2c, intr, 256, 64)
    n = [len(oracle.tile_lists(proj, 256, 64, a, b)[1]) for a, b in [(16, 32), (16, 16), (8, 8)]]
    assert n[0] <= n[1] <= n[2]
    assert (proj["cull"][0] == 0).sum() <= n[0]
