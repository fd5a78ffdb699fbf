"""Pins of the oracle's adjoint (gradients to Gaussians, extrinsic and time offset).

The paper back-propagates the photometric loss to the Gaussian parameters and,
through the input pose, to the calibration (end of Sec. III-B).  The oracle's
analytic adjoint is checked against FP64 central finite differences (h = 1e-6)
of the L1 loss (Eq. 4, L1 part) on small drive scenes with two cameras, and
against closed forms.  Pixels with a threshold decision or an alpha_max kink
within a 1e-2 relative margin are masked on both sides; a coordinate whose
decision signature still changes between +h and -h is rejected.
"""
import numpy as np
import pytest

import oracle
import synth

H_FD = 1e-6
MSET = oracle.Settings(margin=1e-2)


def _setup(seed):
    s = synth.small_drive(seed)
    tgt = oracle.render_scene(s, xi=s.xi_gt, delta=s.delta_gt)["img"]
    base = oracle.render_scene(s, settings=MSET)
    mask = ((base["nflag"] > 0) | (base["kink"] > 0)).astype(np.int8)
    return s, tgt, mask


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_calibration_gradient_matches_fd(seed):
    s, tgt, mask = _setup(seed)
    assert mask.mean() < 0.1
    L, gr, _ = oracle.loss_and_grad(s, tgt, mask=mask)
    checked = 0
    for c in range(s.rig.n):
        for k in range(7):
            vals, sigs = [], []
            for e in (H_FD, -H_FD):
                xi, dl = s.xi.copy(), s.delta.copy()
                if k < 6:
                    xi[c, k] += e
                else:
                    dl[c] += e
                Lv, sg = oracle.fd_loss(s, tgt, s.gauss, xi, dl, mask=mask)
                vals.append(Lv)
                sigs.append(sg)
            if sigs[0] != sigs[1]:
                continue  # the two evaluations straddle a decision: rejected
            fd = (vals[0] - vals[1]) / (2 * H_FD)
            an = gr["xi"][c, k] if k < 6 else gr["delta"][c]
            assert abs(an - fd) <= 1e-6 * abs(fd) + 1e-12, (c, k, an, fd)
            checked += 1
    assert checked >= 12


def test_gaussian_gradient_matches_fd():
    s, tgt, mask = _setup(0)
    L, gr, _ = oracle.loss_and_grad(s, tgt, mask=mask)
    g64 = synth.Gaussians(*[a.astype(np.float64) for a in oracle.gauss64(s.gauss)])
    rng = np.random.default_rng(11)
    vis = np.nonzero(np.abs(gr["opacity"]) > 1e-7)[0]
    # the mean is the LiDAR point the Gaussian is anchored at; its gradient W^T dL/dt (Eq. 2
    # applied to the point, end of Sec. III-B) is pinned here like every other parameter
    params = [("mean", k) for k in range(3)] + [("quat", k) for k in range(4)] + \
             [("scale", k) for k in range(3)] + [("opacity", None)] + [("color", k) for k in range(3)]
    checked = 0
    per_name = {}
    for gi in rng.choice(vis, 24, replace=False):
        for name, k in params:
            vals, sigs = [], []
            for e in (H_FD, -H_FD):
                gg = g64.copy()
                arr = getattr(gg, name)
                if k is None:
                    arr[gi] += e
                else:
                    arr[k, gi] += e
                Lv, sg = oracle.fd_loss(s, tgt, gg, s.xi, s.delta, mask=mask)
                vals.append(Lv)
                sigs.append(sg)
            if sigs[0] != sigs[1]:
                continue
            fd = (vals[0] - vals[1]) / (2 * H_FD)
            an = gr[name][gi] if k is None else gr[name][k, gi]
            # the FD noise floor is about eps * L / h ~ 1e-11 for these losses
            assert abs(an - fd) <= 1e-5 * abs(fd) + 1e-10, (name, k, gi, an, fd)
            checked += 1
            per_name[name] = per_name.get(name, 0) + 1
    assert checked >= 250
    assert per_name.get("mean", 0) >= 60, per_name


def test_color_gradient_is_blend_weight():
    """dC/dc_g = alpha_g T_g (closed form) for a one-hot dL/dimg."""
    s = synth.tiny_scene(1)
    w2c = oracle.pose(s.traj, s.rig, s.xi, s.delta, s.views)[0]
    intr = s.rig.intr
    for (x, y) in [(100, 30), (17, 5), (200, 50)]:
        st = oracle.pixel_stack(s.gauss, w2c[0], intr[0], 256, 64, x, y)
        d = np.zeros((1, 3, 64, 256))
        d[0, 1, y, x] = 1.0
        gr = oracle.grad(s.gauss, w2c, intr, 256, 64, d)
        ids = st[:, 0].astype(int)
        np.testing.assert_allclose(gr["color"][1, ids], st[:, 1] * st[:, 2], rtol=1e-14)
        other = np.setdiff1d(np.arange(s.gauss.n), ids)
        assert np.all(gr["color"][:, other] == 0) and np.all(gr["color"][[0, 2]] == 0)


def test_single_gaussian_opacity_gradient_at_peak():
    """One Gaussian at a pixel centre: C = o c + (1 - o) bg, so dC/do = c - bg."""
    bg = (0.2, 0.1, 0.05)
    st = oracle.Settings(bg=bg)
    c = np.array([0.9, 0.3, 0.6])
    G = synth.Gaussians(np.array([[0.0], [0.0], [5.0]]), np.array([[1.0], [0], [0], [0]]),
                        np.full((3, 1), 0.05), np.array([0.6]), c[:, None].copy())
    I12 = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1).reshape(12)
    for ch in range(3):
        d = np.zeros((1, 3, 32, 32))
        d[0, ch, 16, 16] = 1.0
        gr = oracle.grad(G, I12, [100, 100, 16.5, 16.5], 32, 32, d, st)
        assert abs(gr["opacity"][0] - (c[ch] - bg[ch])) < 1e-14
        # at the peak the mean and conic gradients vanish
        assert np.all(np.abs(gr["mean"][:, 0]) < 1e-14)
