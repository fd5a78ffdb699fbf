"""Pins of the oracle's trajectory, Eq. (1) and Eq. (2) and their adjoint.

Sec. III-A: the LiDAR trajectory interpolates translation linearly and rotation
by SLERP; the camera pose is T_L(t + delta) * T_cam->LiDAR (Eq. 1) and the
world->camera transform is its inverse (Eq. 2).  The pins below use independent
closed forms (Shoemake's sine-weighted SLERP, matrix inverse, scipy rotation
vectors) rather than the oracle's own Exp/Log formulation.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))


def shoemake_slerp(q0, q1, u):
    q0 = q0 / np.linalg.norm(q0)
    q1 = q1 / np.linalg.norm(q1)
    d = float(np.dot(q0, q1))
    if d < 0:
        q1, d = -q1, -d
    th = math.acos(min(1.0, d))
    if th < 1e-12:
        return q0
    return (math.sin((1 - u) * th) * q0 + math.sin(u * th) * q1) / math.sin(th)


def qmat(q):
    w, x, y, z = q
    return Rotation.from_quat([x, y, z, w]).as_matrix()


def one_view_rig():
    return synth.Rig(np.eye(3)[None].copy(), np.zeros((1, 3)), np.array([[100.0, 100.0, 50.0, 50.0]]), 100, 100)


def lidar_pose_from_w2c(w2c):
    """With an identity extrinsic the camera pose equals the LiDAR pose: invert [W|w]."""
    M = np.eye(4)
    M[:3, :] = w2c.reshape(3, 4)
    return np.linalg.inv(M)


def test_slerp_matches_shoemake_random():
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.normal(size=(2, 4))
        p = rng.normal(size=(2, 3))
        # keep the two knots within 170 degrees so the arc is well defined
        if abs(np.dot(q[0] / np.linalg.norm(q[0]), q[1] / np.linalg.norm(q[1]))) < 0.05:
            continue
        u = rng.uniform(0, 1)
        traj = synth.Trajectory(np.array([0.0, 2.0]), q, p)
        views = synth.Views(np.zeros(1, np.int32), np.array([2.0 * u]))
        w2c, seg, uu = oracle.pose(traj, one_view_rig(), np.zeros((1, 6)), np.zeros(1), views)
        T = lidar_pose_from_w2c(w2c[0])
        q_ref = shoemake_slerp(q[0], q[1], u)
        np.testing.assert_allclose(T[:3, :3], qmat(q_ref), atol=1e-12)
        np.testing.assert_allclose(T[:3, 3], (1 - u) * p[0] + u * p[1], atol=1e-12)
        assert seg[0] == 0 and abs(uu[0] - u) < 1e-15


def test_golden_slerp_and_lerp():
    g = GOLD["slerp_z90_half"]
    gl = GOLD["lerp_translation"]
    traj = synth.Trajectory(np.array([0.0, 1.0]), np.array([g["q0"], g["q1"]]), np.array([gl["p0"], gl["p1"]]))
    for u, qexp, pexp in [(g["u"], g["expected_q"], None), (gl["u"], None, gl["expected_p"])]:
        views = synth.Views(np.zeros(1, np.int32), np.array([u]))
        w2c, _, _ = oracle.pose(traj, one_view_rig(), np.zeros((1, 6)), np.zeros(1), views)
        T = lidar_pose_from_w2c(w2c[0])
        if qexp is not None:
            np.testing.assert_allclose(T[:3, :3], qmat(np.array(qexp)), atol=1e-12)
        if pexp is not None:
            np.testing.assert_allclose(T[:3, 3], pexp, atol=1e-12)


def test_fixed_axis_rotation_is_linear_in_u():
    axis = np.array([1.0, 2.0, -0.5])
    axis /= np.linalg.norm(axis)
    theta = 1.3
    q1 = np.r_[math.cos(theta / 2), math.sin(theta / 2) * axis]
    traj = synth.Trajectory(np.array([0.0, 0.1]), np.array([[1.0, 0, 0, 0], q1]), np.zeros((2, 3)))
    for u in (0.0, 0.25, 0.5, 0.9):
        views = synth.Views(np.zeros(1, np.int32), np.array([0.1 * u]))
        w2c, _, _ = oracle.pose(traj, one_view_rig(), np.zeros((1, 6)), np.zeros(1), views)
        R = lidar_pose_from_w2c(w2c[0])[:3, :3]
        rv = Rotation.from_matrix(R).as_rotvec()
        np.testing.assert_allclose(rv, u * theta * axis, atol=1e-12)


def test_knots_and_segments():
    traj = synth.scenes._drive_trajectory(n_knots=11)
    rig = one_view_rig()
    for k in range(10):
        views = synth.Views(np.zeros(1, np.int32), np.array([traj.t[k]]))
        w2c, seg, u = oracle.pose(traj, rig, np.zeros((1, 6)), np.zeros(1), views)
        T = lidar_pose_from_w2c(w2c[0])
        np.testing.assert_allclose(T[:3, :3], qmat(traj.q[k]), atol=1e-12)
        np.testing.assert_allclose(T[:3, 3], traj.p[k], atol=1e-9)
        assert seg[0] == k and u[0] == 0.0  # a knot starts its right segment
    # the last knot is the end of the last segment
    views = synth.Views(np.zeros(1, np.int32), np.array([traj.t[-1]]))
    _, seg, u = oracle.pose(traj, rig, np.zeros((1, 6)), np.zeros(1), views)
    assert seg[0] == 9 and abs(u[0] - 1.0) < 1e-12


def test_eq1_eq2_with_extrinsic_and_offset():
    rng = np.random.default_rng(3)
    traj = synth.scenes._arc_trajectory(6)
    R0 = Rotation.random(2, random_state=1).as_matrix()
    t0 = rng.normal(size=(2, 3))
    rig = synth.Rig(R0, t0, np.array([[100.0, 100, 50, 50]] * 2), 100, 100)
    xi = rng.normal(scale=0.2, size=(2, 6))
    delta = np.array([0.031, -0.017])
    views = synth.Views(np.array([0, 1, 1], np.int32), np.array([0.12, 0.2, 0.33]))
    w2c, _, _ = oracle.pose(traj, rig, xi, delta, views)
    for v in range(3):
        c = views.cam[v]
        s = views.t[v] + delta[c]
        k = int(np.searchsorted(traj.t, s, side="right") - 1)
        u = (s - traj.t[k]) / (traj.t[k + 1] - traj.t[k])
        TL = np.eye(4)
        TL[:3, :3] = qmat(shoemake_slerp(traj.q[k], traj.q[k + 1], u))
        TL[:3, 3] = (1 - u) * traj.p[k] + u * traj.p[k + 1]
        Te = np.eye(4)
        Te[:3, :3] = R0[c] @ Rotation.from_rotvec(xi[c, 3:]).as_matrix()
        Te[:3, 3] = t0[c] + xi[c, :3]
        ref = np.linalg.inv(TL @ Te)[:3, :]
        np.testing.assert_allclose(w2c[v].reshape(3, 4), ref, atol=1e-12)


def _fd_pose_grads(traj, rig, xi, delta, views, G, h=1e-6):
    dxi = np.zeros_like(xi)
    dd = np.zeros_like(delta)
    for c in range(xi.shape[0]):
        for k in range(7):
            vals = []
            for e in (h, -h):
                x2, d2 = xi.copy(), delta.copy()
                if k < 6:
                    x2[c, k] += e
                else:
                    d2[c] += e
                w, _, _ = oracle.pose(traj, rig, x2, d2, views)
                vals.append(float((w * G).sum()))
            g = (vals[0] - vals[1]) / (2 * h)
            if k < 6:
                dxi[c, k] = g
            else:
                dd[c] = g
    return dxi, dd


@pytest.mark.parametrize("phi_scale", [0.3, 1e-8])
def test_pose_adjoint_matches_fd(phi_scale):
    """pose_bwd of a random linear functional of W2C equals FP64 central differences.

    phi_scale = 1e-8 exercises the small-angle branch of the right Jacobian."""
    rng = np.random.default_rng(5)
    traj = synth.scenes._arc_trajectory(8)
    rig = synth.Rig(Rotation.random(2, random_state=2).as_matrix(), rng.normal(size=(2, 3)),
                    np.array([[100.0, 100, 50, 50]] * 2), 100, 100)
    xi = np.concatenate([rng.normal(size=(2, 3)), phi_scale * rng.normal(size=(2, 3))], axis=1)
    delta = np.array([0.043, 0.021])
    views = synth.Views(np.array([0, 0, 1, 1], np.int32), np.array([0.11, 0.36, 0.22, 0.51]))
    G = rng.normal(size=(4, 12))
    dxi, dd = oracle.pose_bwd(traj, rig, xi, delta, views, G)
    fxi, fdd = _fd_pose_grads(traj, rig, xi, delta, views, G)
    np.testing.assert_allclose(dxi, fxi, rtol=1e-6, atol=1e-8)
    np.testing.assert_allclose(dd, fdd, rtol=1e-6, atol=1e-8)


def test_constant_velocity_offset_derivative():
    """Straight constant-velocity drive: d(camera centre)/d(delta) = velocity."""
    v = np.array([10.0, -2.0, 0.5])
    ts = np.arange(5) * 0.1
    traj = synth.Trajectory(ts, np.tile([[1.0, 0, 0, 0]], (5, 1)), ts[:, None] * v[None])
    rig = synth.Rig(np.eye(3)[None].copy(), np.array([[0.3, -0.2, 0.1]]),
                    np.array([[100.0, 100, 50, 50]]), 100, 100)
    xi = np.zeros((1, 6))
    delta = np.array([0.02])
    views = synth.Views(np.zeros(1, np.int32), np.array([0.17]))
    w2c, _, _ = oracle.pose(traj, rig, xi, delta, views)
    W = w2c[0].reshape(3, 4)[:, :3]
    w = w2c[0].reshape(3, 4)[:, 3]
    for a in np.eye(3):
        # L = a . c with c = -W^T w (Eq. 2 inverted); dL/dW_ij = -a_j w_i, dL/dw_i = -(W a)_i
        G = np.zeros((3, 4))
        G[:, :3] = -np.outer(w, a)
        G[:, 3] = -(W @ a)
        _, dd = oracle.pose_bwd(traj, rig, xi, delta, views, G.reshape(1, 12))
        assert abs(dd[0] - a @ v) < 1e-10
