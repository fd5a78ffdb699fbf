"""Pins of the oracle's projection: Eq. (2), Eq. (3) and the EWA projection.

Eq. (3) rotates the Gaussian rotation into the camera frame; the oracle uses the
equivalent covariance form W Sigma W^T, checked here against the quaternion
composition.  The EWA 2-D covariance is checked against closed forms and a
numerical Jacobian of the pinhole projection.
"""
import json
import math
import os
from fractions import Fraction

import numpy as np
from scipy.spatial.transform import Rotation

import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
S = oracle.Settings()


def w2c_of(R, t):
    return np.concatenate([R, t[:, None]], axis=1).reshape(12)


def cov_from(q_wxyz, s):
    R = Rotation.from_quat([q_wxyz[1], q_wxyz[2], q_wxyz[3], q_wxyz[0]]).as_matrix()
    return R @ np.diag(np.asarray(s) ** 2) @ R.T


def test_eq3_equals_rotated_quaternion():
    rng = np.random.default_rng(0)
    for _ in range(30):
        Rw = Rotation.random(random_state=int(rng.integers(1 << 30)))
        t = rng.normal(size=3)
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        s = np.exp(rng.normal(size=3) - 2)
        x = np.array([0.1, -0.2, 5.0]) - t  # keep the mean in front of the camera
        x = Rw.inv().apply(x)
        p = oracle.project_one(x, q, s, 0.9, w2c_of(Rw.as_matrix(), t), [100, 100, 50, 50], 100, 100)
        # Eq. (3): camera-frame rotation is R^-1 r, here as quaternion composition W * r
        rc = Rw * Rotation.from_quat([q[1], q[2], q[3], q[0]])
        qc = rc.as_quat()
        Sc_ref = cov_from([qc[3], qc[0], qc[1], qc[2]], s)
        np.testing.assert_allclose(p["Sc"], Sc_ref, atol=1e-14 * max(1, np.abs(Sc_ref).max()))
        np.testing.assert_allclose(p["t"], Rw.as_matrix() @ x + t, atol=1e-12)


def test_onaxis_isotropic_closed_form():
    g = GOLD["onaxis_isotropic"]
    f, s, z = g["f"], g["s"], g["z"]
    p = oracle.project_one([0, 0, z], [1, 0, 0, 0], [s, s, s], 0.8, w2c_of(np.eye(3), np.zeros(3)),
                           [f, f, 64, 32], 128, 64)
    np.testing.assert_allclose(p["S2"], [g["expected_S2_diag"], 0.0, g["expected_S2_diag"]], rtol=1e-14)
    np.testing.assert_allclose(p["mu"], [64, 32], atol=1e-13)
    np.testing.assert_allclose(p["Q"], [1 / 16.3, 0, 1 / 16.3], rtol=1e-14)


def test_jacobian_matches_numerical_pinhole_derivative():
    rng = np.random.default_rng(1)
    fx, fy, cx, cy = 300.0, 280.0, 160.0, 90.0

    def proj(t):
        return np.array([fx * t[0] / t[2] + cx, fy * t[1] / t[2] + cy])

    for _ in range(20):
        t = np.array([rng.uniform(-2, 2), rng.uniform(-1, 1), rng.uniform(3, 9)])
        p = oracle.project_one(t, [1, 0, 0, 0], [0.1, 0.1, 0.1], 0.8, w2c_of(np.eye(3), np.zeros(3)),
                               [fx, fy, cx, cy], 320, 180)
        assert p["clx"] == 0 and p["cly"] == 0
        Jn = np.zeros((2, 3))
        h = 1e-6
        for k in range(3):
            e = np.zeros(3)
            e[k] = h
            Jn[:, k] = (proj(t + e) - proj(t - e)) / (2 * h)
        np.testing.assert_allclose(p["J"], Jn, rtol=1e-7, atol=1e-7)
        # and the 2-D covariance is J Sc J^T + eps I
        S2 = Jn @ p["Sc"] @ Jn.T + S.eps2d * np.eye(2)
        np.testing.assert_allclose(p["S2"], [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-6)


def test_guard_band_clamps_jacobian_only():
    # a mean far to the left: x/z = -3 is outside the guard band (-cx - 0.15 W)/fx
    p = oracle.project_one([-15.0, 0.0, 5.0], [1, 0, 0, 0], [0.5, 0.5, 0.5], 0.9,
                           w2c_of(np.eye(3), np.zeros(3)), [100, 100, 50, 50], 100, 100)
    lo = (-50 - 0.15 * 100) / 100
    assert p["clx"] == 1 and p["cly"] == 0
    np.testing.assert_allclose(p["J"][0, 2], -100 * lo / 5.0)
    np.testing.assert_allclose(p["mu"][0], 100 * (-3.0) + 50)  # the mean itself is not clamped


def _round_to_f32(fr):
    """Correctly rounded (nearest, ties to even) float32 of an exact rational."""
    f = np.float32(float(fr))
    cands = [f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - fr),
                                     int(np.frombuffer(np.float32(c).tobytes(), np.uint32)[0]) & 1))
    return np.float32(best)


def test_depth32_is_the_exact_fma_chain():
    rng = np.random.default_rng(2)
    for _ in range(200):
        R = Rotation.random(random_state=int(rng.integers(1 << 30))).as_matrix()
        t = rng.normal(scale=50, size=3)
        x = rng.normal(scale=60, size=3).astype(np.float32).astype(np.float64)
        w2c = w2c_of(R, t)
        p = oracle.project_one(x, [1, 0, 0, 0], [0.1] * 3, 0.9, w2c, [100, 100, 50, 50], 100, 100)
        a = [np.float32(w2c[8 + k]) for k in range(4)]
        acc = a[3]
        for k in (2, 1, 0):  # fmaf(a0, x0, fmaf(a1, x1, fmaf(a2, x2, a3)))
            acc = _round_to_f32(Fraction(float(a[k])) * Fraction(float(np.float32(x[k]))) + Fraction(float(acc)))
        assert np.float32(p["depth32"]) == acc


def test_culls():
    I = w2c_of(np.eye(3), np.zeros(3))
    intr = [100, 100, 50, 50]
    args = dict(w2c=I, intr=intr, W=100, H=100)
    cull = lambda x, q=(1, 0, 0, 0), s=(0.1, 0.1, 0.1), o=0.9: int(oracle.project_one(x, q, s, o, **args)["cull"])
    assert cull([0, 0, 5.0]) == 0
    assert cull([0, 0, 0.2]) == 1            # depth32 <= near_z
    assert cull([0, 0, -3.0]) == 1           # behind the camera
    assert cull([0, 0, 300.0]) == 2          # beyond the far plane
    assert cull([0, 0, 5.0], o=0.003) == 4   # opacity below alpha_min
    assert cull([0, 0, 5.0], q=(0, 0, 0, 0)) == 8
    assert cull([40.0, 0, 5.0]) == 16        # footprint entirely off screen
    assert cull([np.nan, 0, 5.0]) == 32


def test_footprint_is_the_opacity_aware_ellipse_box():
    o = 0.6
    p = oracle.project_one([0.3, -0.1, 4.0], [0.9, 0.2, -0.3, 0.1], [0.3, 0.05, 0.12], o,
                           w2c_of(np.eye(3), np.zeros(3)), [200, 200, 100, 60], 200, 120)
    k = math.sqrt(2 * math.log(o / S.alpha_min))
    np.testing.assert_allclose(p["rad"], [k * math.sqrt(p["S2"][0]), k * math.sqrt(p["S2"][2])], rtol=1e-14)
    # dense check: every pixel centre with alpha >= alpha_min lies inside the rect
    Q = p["Q"]
    ys, xs = np.mgrid[0:120, 0:200]
    dx, dy = xs + 0.5 - p["mu"][0], ys + 0.5 - p["mu"][1]
    alpha = o * np.exp(-0.5 * (Q[0] * dx * dx + 2 * Q[1] * dx * dy + Q[2] * dy * dy))
    inside = (xs >= p["rect"][0]) & (xs <= p["rect"][1]) & (ys >= p["rect"][2]) & (ys <= p["rect"][3])
    assert (alpha >= S.alpha_min).sum() > 50
    assert not np.any((alpha >= S.alpha_min) & ~inside)
