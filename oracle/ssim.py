"""D-SSIM term of the photometric loss (paper Eq. 4: the loss of the original 3DGS
work) -- test infrastructure only, plain PyTorch CPU float64.

SSIM with an 11 x 11 Gaussian window (sigma 1.5, normalised), zero padding, per
channel, C1 = 0.01^2, C2 = 0.03^2; the loss term is weight * (1 - mean SSIM) over
every view, channel and pixel of the rows [roi_y0, H) (the image is cropped to the
region of interest first, Sec. III-C).  The gradient is torch autograd of that
definition.
"""
from __future__ import annotations

import numpy as np

C1, C2 = 0.01 ** 2, 0.03 ** 2
RADIUS, SIGMA = 5, 1.5

__all__ = ["window_1d", "ssim_map", "dssim", "C1", "C2", "RADIUS", "SIGMA"]


def window_1d():
    i = np.arange(-RADIUS, RADIUS + 1, dtype=np.float64)
    g = np.exp(-(i * i) / (2.0 * SIGMA * SIGMA))
    return g / g.sum()


def _maps(x, y):
    import torch
    import torch.nn.functional as F
    g = torch.as_tensor(window_1d(), dtype=torch.float64)
    w = torch.outer(g, g).expand(3, 1, 2 * RADIUS + 1, 2 * RADIUS + 1).contiguous()

    def conv(t):
        return F.conv2d(t, w, padding=RADIUS, groups=3)

    mu1, mu2 = conv(x), conv(y)
    s11 = conv(x * x) - mu1 * mu1
    s22 = conv(y * y) - mu2 * mu2
    s12 = conv(x * y) - mu1 * mu2
    return ((2 * mu1 * mu2 + C1) * (2 * s12 + C2)) / ((mu1 * mu1 + mu2 * mu2 + C1) * (s11 + s22 + C2))


def ssim_map(img, target, roi_y0=0):
    """SSIM map [V,3,H-roi_y0,W] of the cropped images (float64 numpy)."""
    import torch
    x = torch.as_tensor(np.ascontiguousarray(img[:, :, roi_y0:]), dtype=torch.float64)
    y = torch.as_tensor(np.ascontiguousarray(target[:, :, roi_y0:]), dtype=torch.float64)
    return _maps(x, y).numpy()


def dssim(img, target, roi_y0=0, weight=1.0):
    """weight * (1 - mean SSIM) over the rows [roi_y0, H) and its gradient [V,3,H,W] w.r.t. img."""
    import torch
    x = torch.tensor(np.ascontiguousarray(img[:, :, roi_y0:]), dtype=torch.float64, requires_grad=True)
    y = torch.as_tensor(np.ascontiguousarray(target[:, :, roi_y0:]), dtype=torch.float64)
    L = weight * (1.0 - _maps(x, y).mean())
    L.backward()
    grad = np.zeros(np.shape(img), np.float64)
    grad[:, :, roi_y0:] = x.grad.numpy()
    return float(L.item()), grad
