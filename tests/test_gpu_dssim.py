"""GPU parity of the D-SSIM term (Eq. 4) against the float64 PyTorch oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2403_11577_amd import binding as B
from paper_2403_11577_amd import pipeline as pl

from gpu_util import say

pytestmark = pytest.mark.gpu


def _smooth(rng, V, H, W):
    """Images with structure at several scales (so SSIM is far from 0 and 1)."""
    yy, xx = np.mgrid[0:H, 0:W] / max(H, W)
    out = np.zeros((V, 3, H, W))
    for v in range(V):
        for c in range(3):
            f = rng.uniform(2, 12, size=(4, 2))
            ph = rng.uniform(0, 6.3, size=4)
            out[v, c] = 0.5 + 0.12 * sum(np.sin(f[k, 0] * xx * 6.3 + f[k, 1] * yy * 6.3 + ph[k]) for k in range(4))
    return np.clip(out + rng.normal(0, 0.03, size=out.shape), 0, 1)


def _gpu_dssim(img, tgt, roi, weight, base=None):
    V, _, H, W = img.shape
    it = torch.as_tensor(img.astype(np.float32), device="cuda")
    tt = torch.as_tensor(tgt.astype(np.float32), device="cuda")
    ws = torch.empty(B.splat_dssim_workspace_size(V, W, H, roi), dtype=torch.uint8, device="cuda")
    d = torch.zeros_like(it) if base is None else base
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.splat_dssim_loss_grad(it, tt, ws, d, loss, roi_y0=roi, weight=weight)
    torch.cuda.synchronize()
    return float(loss.item()), d.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("kind", ["random", "smooth"])
# tile counts (32 x 21 output tiles per view and channel): 24, 24, 24, 9, 3 (fewer workgroups than
# XCDs: one sequence of tiles) and 18 (a grid of 16 workgroups: uneven ranges per XCD)
@pytest.mark.parametrize("shape, roi", [((2, 37, 50), 0), ((2, 37, 50), 11), ((1, 70, 97), 35), ((3, 9, 13), 2),
                                        ((1, 9, 13), 0), ((1, 30, 70), 0)])
def test_dssim_vs_oracle(kind, shape, roi):
    say(f"case: dssim {kind} shape={shape} roi={roi}")
    V, H, W = shape
    rng = np.random.default_rng(H * W + roi)
    if kind == "random":
        img, tgt = rng.uniform(size=(V, 3, H, W)), rng.uniform(size=(V, 3, H, W))
    else:
        img, tgt = _smooth(rng, V, H, W), _smooth(rng, V, H, W)
    img32, tgt32 = img.astype(np.float32).astype(np.float64), tgt.astype(np.float32).astype(np.float64)
    L, g = _gpu_dssim(img32, tgt32, roi, 0.2)
    Lr, gr = oracle.dssim(img32, tgt32, roi_y0=roi, weight=0.2)
    say(f"  loss {L:.8f} vs {Lr:.8f}, max|g - ref| / max|ref| = {np.abs(g - gr).max() / np.abs(gr).max():.2e}")
    assert L == pytest.approx(Lr, rel=1e-7, abs=1e-12)
    assert np.all(g[:, :, :roi] == 0.0)
    np.testing.assert_allclose(g, gr, rtol=0, atol=2e-6 * np.abs(gr).max())


def test_photometric_loss_is_weighted_l1_plus_dssim():
    say("case: L_photo = 0.8 L1 + 0.2 D-SSIM")
    rng = np.random.default_rng(5)
    V, H, W, roi = 2, 40, 64, 20
    img = _smooth(rng, V, H, W).astype(np.float32)
    tgt = _smooth(rng, V, H, W).astype(np.float32)
    it, tt = torch.as_tensor(img, device="cuda"), torch.as_tensor(tgt, device="cuda")
    d = torch.empty_like(it)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    B.splat_l1_loss_grad(it, tt, None, d, loss, roi_y0=roi, weight=0.8)
    Ls, gs = _gpu_dssim(img.astype(np.float64), tgt.astype(np.float64), roi, 0.2, base=d)
    L1r, g1r = oracle.l1_loss(img.astype(np.float64), tgt.astype(np.float64), roi_y0=roi)
    Lsr, gsr = oracle.dssim(img.astype(np.float64), tgt.astype(np.float64), roi_y0=roi, weight=0.2)
    assert float(loss.item()) + Ls == pytest.approx(0.8 * L1r + Lsr, rel=1e-7)
    ref = 0.8 * g1r + gsr
    np.testing.assert_allclose(gs, ref, rtol=0, atol=2e-6 * np.abs(ref).max())


def test_dssim_full_size_views():
    say("case: dssim 4 x 1408 x 376, bottom half")
    rng = np.random.default_rng(6)
    V, H, W, roi = 4, 376, 1408, 188
    img, tgt = _smooth(rng, V, H, W), _smooth(rng, V, H, W)
    img32, tgt32 = img.astype(np.float32).astype(np.float64), tgt.astype(np.float32).astype(np.float64)
    L, g = _gpu_dssim(img32, tgt32, roi, 0.2)
    Lr, gr = oracle.dssim(img32, tgt32, roi_y0=roi, weight=0.2)
    say(f"  loss {L:.8f} vs {Lr:.8f}")
    assert L == pytest.approx(Lr, rel=1e-7)
    np.testing.assert_allclose(g, gr, rtol=0, atol=2e-6 * np.abs(gr).max())
