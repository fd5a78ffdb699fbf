"""Pins of the oracle's compositing (the EWA splatting function Phi, Eq. 5).

Closed forms (one, two and N identical Gaussians), invariants (weights sum to
1 - T_final, non-increasing transmittance, rigid-motion invariance), the
alpha_min / alpha_max / t_min readings, brute force == AABB-pruned bitwise, and
the threshold-margin alternatives.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
I12 = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)


def gauss(means, opac, colors, scale=0.05, quat=None):
    n = len(opac)
    q = np.tile([[1.0], [0.0], [0.0], [0.0]], (1, n)) if quat is None else np.asarray(quat, np.float64)
    return synth.Gaussians(np.asarray(means, np.float64).T.copy(), q,
                           np.full((3, n), scale, np.float64), np.asarray(opac, np.float64),
                           np.asarray(colors, np.float64).T.copy())


def centred(z, W=32, H=32, f=100.0):
    # a Gaussian at camera (0,0,z) projects to (cx, cy); put cx, cy at a pixel centre
    return [f, f, W / 2 + 0.5, H / 2 + 0.5]


def test_single_gaussian_peak():
    g = GOLD["single_gaussian_peak"]
    st = oracle.Settings(bg=tuple(g["bg"]))
    G = gauss([[0, 0, 5.0]], [g["opacity"]], [g["color"]])
    r = oracle.render(G, I12, centred(5.0), 32, 32, st)
    np.testing.assert_allclose(r["img"][0, :, 16, 16], g["expected_C"], atol=1e-15)
    assert abs(r["T"][0, 16, 16] - g["expected_T"]) < 1e-15
    assert r["last"][0, 16, 16] == 0
    assert r["last"][0, 0, 0] == -1 and r["T"][0, 0, 0] == 1.0
    np.testing.assert_allclose(r["img"][0, :, 0, 0], g["bg"])


def test_two_gaussians_front_to_back():
    g = GOLD["two_gaussians"]
    G = gauss([[0, 0, 5.0], [0, 0, 6.0]], g["alpha"], g["color"])
    intr = [100, 100, 16.5, 16.5]
    # the second Gaussian is farther; scale it so both peak at the same pixel centre
    r = oracle.render(G, I12, intr, 32, 32)
    np.testing.assert_allclose(r["img"][0, :, 16, 16], g["expected_C"], atol=1e-15)
    assert abs(r["T"][0, 16, 16] - g["expected_T"]) < 1e-15
    assert r["last"][0, 16, 16] == 1
    # reversing the depths reverses the order
    G2 = gauss([[0, 0, 6.0], [0, 0, 5.0]], g["alpha"], g["color"])
    r2 = oracle.render(G2, I12, intr, 32, 32)
    np.testing.assert_allclose(r2["img"][0, :, 16, 16], [0.5 * 0.2, 0.8, 0.0], atol=1e-15)
    assert r2["last"][0, 16, 16] == 0


def test_termination_count_of_identical_gaussians():
    g = GOLD["termination_count"]
    n = 30
    G = gauss([[0, 0, 5.0 + 0.01 * i] for i in range(n)], [g["alpha"]] * n, [[1, 1, 1]] * n)
    r = oracle.render(G, I12, [100, 100, 16.5, 16.5], 32, 32)
    st = oracle.pixel_stack(G, I12, [100, 100, 16.5, 16.5], 32, 32, 16, 16)
    assert len(st) == g["expected_blended"]
    assert r["last"][0, 16, 16] == g["expected_blended"] - 1
    assert abs(r["T"][0, 16, 16] - 0.5 ** g["expected_blended"]) < 1e-15


def test_alpha_max_clamp_and_alpha_min_cull():
    G = gauss([[0, 0, 5.0], [0, 0, 6.0]], [0.999, 0.5], [[1, 0, 0], [0, 1, 0]])
    r = oracle.render(G, I12, [100, 100, 16.5, 16.5], 32, 32)
    assert abs(r["T"][0, 16, 16] - 0.01 * 0.5) < 1e-15
    np.testing.assert_allclose(r["img"][0, :, 16, 16], [0.99, 0.01 * 0.5, 0], atol=1e-15)
    # a Gaussian with opacity below alpha_min never contributes anywhere
    G = gauss([[0, 0, 5.0]], [1 / 255 * 0.999], [[1, 1, 1]], scale=1.0)
    r = oracle.render(G, I12, [100, 100, 16.5, 16.5], 32, 32)
    assert np.all(r["img"] == 0) and np.all(r["last"] == -1) and r["stats"]["visible"] == 0


@pytest.mark.parametrize("seed", [0, 1])
def test_weights_sum_to_one_minus_T(seed):
    s = synth.tiny_scene(seed)
    g = s.gauss.copy()
    g.color[:] = 1.0
    r = oracle.render_scene(s, g)
    for c in range(3):
        np.testing.assert_allclose(r["img"][0, c], 1.0 - r["T"][0], atol=1e-14)
    assert np.all(r["T"] >= oracle.Settings().t_min) and np.all(r["T"] <= 1.0)


def test_transmittance_non_increasing_and_stack_consistent():
    s = synth.tiny_scene(0)
    w2c = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)[0][0]
    intr = s.rig.intr[0]
    r = oracle.render_scene(s)
    rng = np.random.default_rng(0)
    for _ in range(40):
        x, y = int(rng.integers(256)), int(rng.integers(64))
        st = oracle.pixel_stack(s.gauss, w2c, intr, 256, 64, x, y)
        if len(st) == 0:
            assert r["last"][0, y, x] == -1
            continue
        T = st[:, 2]
        assert np.all(np.diff(T) <= 0)
        assert st[-1, 0] == r["last"][0, y, x]
        assert abs(T[-1] * (1 - st[-1, 1]) - r["T"][0, y, x]) < 1e-15
        assert np.all(st[:, 1] >= oracle.Settings().alpha_min)


@pytest.mark.parametrize("maker", ["tiny", "small_drive"])
def test_brute_force_equals_pruned_bitwise(maker):
    s = synth.tiny_scene(3) if maker == "tiny" else synth.small_drive(1)
    a = oracle.render_scene(s, pruned=False)
    b = oracle.render_scene(s, pruned=True)
    assert np.array_equal(a["img"], b["img"])
    assert np.array_equal(a["T"], b["T"])
    assert np.array_equal(a["last"], b["last"])
    assert a["hash"] == b["hash"]
    assert b["stats"]["evaluated"] < a["stats"]["evaluated"]


def test_rigid_motion_invariance():
    """Moving the whole world (trajectory, points, Gaussian rotations) rigidly leaves the images unchanged."""
    from scipy.spatial.transform import Rotation
    s = synth.small_drive(2)
    g = s.gauss.copy()
    g64 = synth.Gaussians(*[a.astype(np.float64) for a in oracle.gauss64(g)])
    base = oracle.render_scene(s, g64)
    rng = np.random.default_rng(7)
    Rg = Rotation.random(random_state=4)
    tg = rng.normal(size=3) * 3
    # depth32 rounds the moved means to float32, so near depth ties may swap; the image stays close
    mean = Rg.apply(g64.mean.T) + tg
    g2 = g64.copy()
    g2.mean = mean.T.copy()
    qs = Rotation.from_quat(np.c_[g64.quat[1:].T, g64.quat[0]])
    qn = (Rg * qs).as_quat()
    g2.quat = np.c_[qn[:, 3], qn[:, :3]].T.copy()
    traj = synth.Trajectory(s.traj.t.copy(), s.traj.q.copy(), Rg.apply(s.traj.p) + tg)
    qt = (Rg * Rotation.from_quat(np.c_[s.traj.q[:, 1:], s.traj.q[:, 0]])).as_quat()
    traj.q = np.c_[qt[:, 3], qt[:, :3]]
    s2 = synth.Scene(s.name, g2, traj, s.rig, s.views, s.xi, s.delta, s.xi_gt, s.delta_gt)
    moved = oracle.render_scene(s2)
    # depth order is the float32 depth, which rounding may permute for near ties; the image is still close
    assert np.abs(moved["img"] - base["img"]).max() < 1e-6
    assert (moved["last"] != base["last"]).mean() < 1e-3


def test_margin_alternatives():
    """A Gaussian whose alpha sits at alpha_min within the margin yields two valid outcomes."""
    amin = oracle.Settings().alpha_min
    # choose opacity and offset so that alpha at the pixel centre is alpha_min * (1 + 1e-6)
    G = gauss([[0, 0, 5.0], [0, 0, 6.0]], [0.5, 0.8], [[1, 0, 0], [0, 0, 1]], scale=0.05)
    intr = [100, 100, 16.5, 16.5]
    p = oracle.project_one([0, 0, 5.0], [1, 0, 0, 0], [0.05] * 3, 0.5, I12, intr, 32, 32)
    q = p["Q"][0]
    d = np.sqrt(-2 * np.log(amin * (1 + 1e-6) / 0.5) / q)
    x = 16 + int(np.floor(d))
    frac = d - np.floor(d)
    intr2 = [100, 100, 16.5 - frac, 16.5]  # shift the principal point so pixel x sits at distance d
    r = oracle.render(G, I12, intr2, 32, 32, alternatives=True)
    assert r["nflag"][0, 16, x] == 1
    assert r["nalt"][0, 16, x] == 2
    alts = r["alt"][0, 16, x, :2]
    assert alts[0, 4] != alts[1, 4] or abs(alts[0, 0] - alts[1, 0]) > 1e-4 * amin
    assert r["stats"]["flagged_px"] >= 1
