"""Pins of the D-SSIM oracle (the D-SSIM term of Eq. 4, as in the original 3DGS loss)."""
import numpy as np
import pytest

import oracle
from oracle import ssim as S


def test_window_is_a_normalised_gaussian():
    g = S.window_1d()
    assert g.shape == (11,) and g.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(g, g[::-1]) and g.argmax() == 5
    assert g[6] / g[5] == pytest.approx(np.exp(-1.0 / (2 * 1.5 ** 2)), rel=1e-14)


def test_identical_images_have_ssim_one_and_zero_gradient():
    rng = np.random.default_rng(0)
    x = rng.uniform(size=(2, 3, 20, 23))
    L, g = oracle.dssim(x, x.copy())
    assert L == pytest.approx(0.0, abs=1e-14)
    assert np.abs(g).max() < 1e-12


def test_constant_images_interior_closed_form():
    a, b = 0.3, 0.7
    x = np.full((1, 3, 25, 25), a)
    y = np.full((1, 3, 25, 25), b)
    m = oracle.ssim_map(x, y)
    # a full window (rows/cols 5..19): no variance, mu = a, b
    expect = (2 * a * b + S.C1) / (a * a + b * b + S.C1)
    np.testing.assert_allclose(m[:, :, 5:20, 5:20], expect, rtol=1e-11)  # E[x^2] - mu^2 cancels to ~1e-17
    # at a corner the zero padding shrinks the window sums: not the interior value
    assert abs(m[0, 0, 0, 0] - expect) > 1e-3


def test_ssim_is_symmetric():
    rng = np.random.default_rng(1)
    x, y = rng.uniform(size=(1, 3, 16, 18)), rng.uniform(size=(1, 3, 16, 18))
    np.testing.assert_allclose(oracle.ssim_map(x, y), oracle.ssim_map(y, x), rtol=1e-13)


def test_roi_crops_before_filtering():
    rng = np.random.default_rng(2)
    x, y = rng.uniform(size=(1, 3, 30, 17)), rng.uniform(size=(1, 3, 30, 17))
    roi = 12
    L, g = oracle.dssim(x, y, roi_y0=roi, weight=0.2)
    Lc, gc = oracle.dssim(x[:, :, roi:], y[:, :, roi:], weight=0.2)
    assert L == pytest.approx(Lc, rel=1e-14)
    assert np.all(g[:, :, :roi] == 0.0)
    np.testing.assert_allclose(g[:, :, roi:], gc, rtol=1e-13, atol=1e-18)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    x, y = rng.uniform(size=(1, 3, 14, 15)), rng.uniform(size=(1, 3, 14, 15))
    L, g = oracle.dssim(x, y, weight=0.2)
    h = 1e-6
    for (c, i, j) in [(0, 0, 0), (1, 7, 7), (2, 13, 14), (0, 3, 11), (2, 10, 2)]:
        xp, xm = x.copy(), x.copy()
        xp[0, c, i, j] += h
        xm[0, c, i, j] -= h
        fd = (oracle.dssim(xp, y, weight=0.2)[0] - oracle.dssim(xm, y, weight=0.2)[0]) / (2 * h)
        assert fd == pytest.approx(g[0, c, i, j], rel=1e-6, abs=1e-12)
