"""Pins of the image-quality metrics (PSNR, SSIM of Wang et al. 2004) that
every reported quality figure comes from: special cases with known values and
a brute-force SSIM written window by window."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2407_19097_amd import metrics  # noqa: E402


def t(a):
    return torch.from_numpy(np.asarray(a, np.float32))


def test_psnr_identical_is_infinite():
    a = t(np.random.default_rng(0).random((2, 3, 9, 7)))
    assert torch.isinf(metrics.psnr(a, a)).all()


def test_psnr_known_mse():
    a = torch.zeros((1, 3, 8, 8))
    b = torch.full((1, 3, 8, 8), 0.1)
    # MSE 0.01 -> 20 dB; MSE 0.25 -> 6.0206 dB
    assert abs(metrics.psnr(a, b).item() - 20.0) < 1e-4
    c = torch.zeros((1, 3, 8, 8))
    c[:, :, :, :4] = 0.5
    d = torch.zeros((1, 3, 8, 8))
    d[:, :, :, 4:] = 0.5
    assert abs(metrics.psnr(c, d).item() - 10 * math.log10(1 / 0.25)) < 1e-4
    # values outside [0, 1] count as clamped
    assert abs(metrics.psnr(a - 1.0, b).item() - 20.0) < 1e-4


def test_ssim_identical_is_one():
    a = t(np.random.default_rng(1).random((2, 3, 20, 17)))
    np.testing.assert_allclose(metrics.ssim(a, a).numpy(), 1.0, atol=1e-6)


def test_ssim_constant_images_closed_form():
    """Zero variance everywhere: SSIM = (2 a b + C1) / (a^2 + b^2 + C1)."""
    a = torch.full((1, 3, 16, 16), 0.5)
    b = torch.full((1, 3, 16, 16), 0.25)
    c1 = 0.01 ** 2
    want = (2 * 0.5 * 0.25 + c1) / (0.25 + 0.0625 + c1)
    assert abs(metrics.ssim(a, b).item() - want) < 1e-5


def test_ssim_matches_brute_force_windows():
    """Per valid 11 x 11 window, the weighted means, variances and covariance
    from a 2-D Gaussian weight table, in float64, averaged over windows and
    channels."""
    rng = np.random.default_rng(2)
    H, W = 18, 15
    A = rng.random((3, H, W))
    B = np.clip(A + 0.2 * rng.standard_normal((3, H, W)), 0, 1)
    x = np.arange(11) - 5.0
    g1 = np.exp(-x * x / (2 * 1.5 * 1.5))
    w2 = np.outer(g1, g1)
    w2 /= w2.sum()
    c1, c2 = 0.01 ** 2, 0.03 ** 2
    vals = []
    for c in range(3):
        for i in range(H - 10):
            for j in range(W - 10):
                pa, pb = A[c, i:i + 11, j:j + 11], B[c, i:i + 11, j:j + 11]
                ma, mb = (w2 * pa).sum(), (w2 * pb).sum()
                va = (w2 * (pa - ma) ** 2).sum()
                vb = (w2 * (pb - mb) ** 2).sum()
                cab = (w2 * (pa - ma) * (pb - mb)).sum()
                vals.append(((2 * ma * mb + c1) * (2 * cab + c2)) / ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    want = float(np.mean(vals))
    got = metrics.ssim(t(A[None]), t(B[None])).item()
    assert 0.2 < want < 0.99
    assert abs(got - want) < 2e-5, (got, want)
