"""Image-quality metrics used to judge the post-process against the splat
renderer (the paper reports PSNR and SSIM, Sec. 4.1).

PSNR = 10 log10(1 / MSE) for images in [0, 1], over all channels.
SSIM after Wang et al. (2004): 11 x 11 Gaussian window with sigma 1.5,
K1 = 0.01, K2 = 0.03, dynamic range 1, computed per channel on the valid
region and averaged.  Batched torch tensors [N, 3, H, W] in, one value per
image out.
"""
from __future__ import annotations

import math


def psnr(a, b):
    d = (a.double() - b.double()) ** 2
    mse = d.flatten(1).mean(dim=1)
    return 10.0 * (1.0 / mse.clamp_min(1e-20)).log10()


def _gauss(torch, device):
    x = torch.arange(11, dtype=torch.float64, device=device) - 5.0
    g = torch.exp(-(x * x) / (2.0 * 1.5 * 1.5))
    g = g / g.sum()
    return g


def ssim(a, b):
    import torch
    import torch.nn.functional as F
    a = a.double()
    b = b.double()
    n, c, h, w = a.shape
    g = _gauss(torch, a.device)
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
