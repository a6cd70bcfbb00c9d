"""Image-quality metrics used to judge the post-process against the splat
renderer (the paper reports PSNR and SSIM, Sec. 4.1, without defining its
variants).

PSNR = 10 log10(1 / MSE) for images in [0, 1], over all channels (+inf for
identical images).
SSIM after Wang et al. (2004): 11 x 11 Gaussian window with sigma 1.5,
K1 = 0.01, K2 = 0.03, dynamic range 1, computed per channel on the valid
region (no padding) and averaged over pixels and channels.

Batched torch tensors [N, C, H, W] in, one value per image out.  Both run in
fp32 on the tensors' own device (evaluation only, not part of the hot path);
images are clamped to [0, 1] first, as they would be displayed.
"""
from __future__ import annotations

import math


def _prep(a):
    return a.float().clamp(0.0, 1.0)


def psnr(a, b):
    import torch
    d = _prep(a) - _prep(b)
    mse = (d * d).flatten(1).mean(dim=1)
    inf = torch.full_like(mse, math.inf)
    return torch.where(mse > 0, 10.0 * torch.log10(1.0 / mse.clamp_min(1e-30)), inf)


def gaussian_window(torch, device, size=11, sigma=1.5):
    x = torch.arange(size, dtype=torch.float32, device=device) - (size - 1) / 2.0
    g = torch.exp(-(x * x) / (2.0 * sigma * sigma))
    return g / g.sum()


def ssim(a, b):
    import torch
    import torch.nn.functional as F
    a, b = _prep(a), _prep(b)
    n, c, h, w = a.shape
    g = gaussian_window(torch, a.device)
    kx = g.view(1, 1, 1, 11).repeat(c, 1, 1, 1)
    ky = g.view(1, 1, 11, 1).repeat(c, 1, 1, 1)

    def blur(t):
        return F.conv2d(F.conv2d(t, kx, groups=c), ky, groups=c)

    mu_a, mu_b = blur(a), blur(b)
    saa = blur(a * a) - mu_a * mu_a
    sbb = blur(b * b) - mu_b * mu_b
    sab = blur(a * b) - mu_a * mu_b
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    s = ((2 * mu_a * mu_b + c1) * (2 * sab + c2)) / ((mu_a * mu_a + mu_b * mu_b + c1) * (saa + sbb + c2))
    return s.flatten(1).mean(dim=1)
