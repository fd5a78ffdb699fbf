"""Oracle pins for the region of interest (bottom rows only, Sec. III-C image cropping)
and the scale regulariser L_scale of Sec. III-C."""
import numpy as np
import pytest

import oracle
import synth


def _scene():
    return synth.tiny_scene(3, n=400, W=96, H=40, f=60.0)


@pytest.mark.parametrize("pruned", [True, False])
@pytest.mark.parametrize("roi", [20, 23, 39])
def test_roi_render_is_the_cropped_full_render(pruned, roi):
    s = _scene()
    w2c, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    intr = oracle.view_intr(s.rig, s.views)
    bg = (0.25, 0.5, 0.75)
    full = oracle.render(s.gauss, w2c, intr, s.rig.W, s.rig.H, oracle.Settings(bg=bg), pruned=pruned)
    part = oracle.render(s.gauss, w2c, intr, s.rig.W, s.rig.H, oracle.Settings(bg=bg, roi_y0=roi), pruned=pruned)
    # inside the region of interest: bitwise the full render
    assert np.array_equal(part["img"][:, :, roi:], full["img"][:, :, roi:])
    assert np.array_equal(part["T"][:, roi:], full["T"][:, roi:])
    assert np.array_equal(part["last"][:, roi:], full["last"][:, roi:])
    # above it: not rendered
    for c in range(3):
        assert np.all(part["img"][:, c, :roi] == bg[c])
    assert np.all(part["T"][:, :roi] == 1.0) and np.all(part["last"][:, :roi] == -1)
    assert full["last"][:, :roi].max() >= 0  # the rows above do have contributors in the full render


def test_roi_binning_lists_only_tiles_inside_the_region():
    s = _scene()
    w2c, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    intr = oracle.view_intr(s.rig, s.views)
    roi = 21
    pf = oracle.project_all(s.gauss, w2c, intr, s.rig.W, s.rig.H)
    pr = oracle.project_all(s.gauss, w2c, intr, s.rig.W, s.rig.H, oracle.Settings(roi_y0=roi))
    vis_f, vis_r = pf["cull"] == 0, pr["cull"] == 0
    # visible with the region iff the full footprint reaches a row >= roi
    assert np.array_equal(vis_r, vis_f & (pf["rect"][..., 3] >= roi))
    assert np.all(pr["rect"][..., 2][vis_r] == np.maximum(pf["rect"][..., 2][vis_r], roi))
    assert np.array_equal(pr["rect"][..., 3][vis_r], pf["rect"][..., 3][vis_r])


def test_roi_gradient_is_the_full_gradient_with_the_rows_above_zeroed():
    s = _scene()
    w2c, _, _ = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)
    intr = oracle.view_intr(s.rig, s.views)
    roi = 17
    rng = np.random.default_rng(0)
    dimg = rng.normal(size=(s.views.n, 3, s.rig.H, s.rig.W))
    dz = dimg.copy()
    dz[:, :, :roi] = 0.0
    full = oracle.grad(s.gauss, w2c, intr, s.rig.W, s.rig.H, dz)
    part = oracle.grad(s.gauss, w2c, intr, s.rig.W, s.rig.H, dimg, oracle.Settings(roi_y0=roi))
    for k in ("quat", "scale", "opacity", "color", "mean", "w2c"):
        np.testing.assert_allclose(part[k], full[k], rtol=1e-12, atol=1e-15 * max(1.0, np.abs(full[k]).max()))


def test_roi_l1_closed_form():
    rng = np.random.default_rng(1)
    V, H, W, roi, c = 2, 10, 7, 4, 0.125
    target = rng.uniform(size=(V, 3, H, W))
    img = target + c
    img[:, :, :roi] = rng.uniform(size=(V, 3, roi, W))  # anything above the region of interest
    L, g = oracle.l1_loss(img, target, roi_y0=roi)
    assert L == pytest.approx(c, rel=1e-14)
    n = V * 3 * (H - roi) * W
    assert np.all(g[:, :, :roi] == 0.0)
    np.testing.assert_array_equal(g[:, :, roi:], np.full((V, 3, H - roi, W), 1.0 / n))


@pytest.mark.parametrize("s, loss, grad", [
    ((0.3, 0.3, 0.3), 0.0, (0.0, 0.0, 0.0)),           # isotropic: no penalty
    ((1.0, 2.0, 3.0), 2.0, (-1.0, 0.0, 1.0)),          # mean 2: |1-2| + |3-2|
    ((1.0, 1.0, 4.0), 4.0, (-2 / 3, -2 / 3, 4 / 3)),   # mean 2: two below, one above
])
def test_scale_reg_closed_forms(s, loss, grad):
    lam = 1e-3
    L, g = oracle.scale_reg(np.array(s).reshape(3, 1), lam)
    assert L == pytest.approx(lam * loss, abs=1e-18)
    np.testing.assert_allclose(g[:, 0], lam * np.array(grad), atol=1e-18)


def test_scale_reg_gradient_matches_central_differences():
    rng = np.random.default_rng(2)
    s = np.exp(rng.normal(np.log(0.1), 0.5, size=(3, 50)))
    lam, h = 1e-3, 1e-7
    _, g = oracle.scale_reg(s, lam)
    for k in range(3):
        for j in range(0, 50, 7):
            sp, sm = s.copy(), s.copy()
            sp[k, j] += h
            sm[k, j] -= h
            fd = (oracle.scale_reg(sp, lam)[0] - oracle.scale_reg(sm, lam)[0]) / (2 * h)
            assert fd == pytest.approx(g[k, j], rel=1e-6, abs=1e-12)
