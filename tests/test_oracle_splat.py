"""Pins for the CPU Gaussian-splat oracle (the Gaussian renderer of Sec. 4.2:
points as Gaussians, depth-sorted, alpha-blended front to back) against
closed forms: one Gaussian, two overlapping Gaussians, early termination,
tie order, the 3-sigma footprint and culling."""
import math

import numpy as np
import pytest

from oracle import camera as ocam
from oracle import splat as osplat
from paper_2407_19097_amd import scenes

SIG = 1.5


def cam_identity():
    return scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0), fovy_deg=90.0)


def centre64(M, p, W, H):
    Md = M.astype(np.float64).reshape(4, 4)
    c = Md @ np.append(np.asarray(p, np.float64), 1.0)
    return (c[0] / c[3] * 0.5 + 0.5) * W, (0.5 - c[1] / c[3] * 0.5) * H


def alpha(d2, o=1.0):
    a = min(0.99, o * math.exp(-d2 / (2 * SIG * SIG)))
    return a if a >= 1 / 255 else 0.0


def rgb8(cols):
    cols = np.asarray(cols, np.uint8)
    return [np.ascontiguousarray(cols[:, c]) for c in range(3)]


def test_single_gaussian_closed_form():
    W, H = 24, 20
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    p = (0.13, -0.07, -1.0)
    img = osplat.splat(*[np.array([v], np.float32) for v in p], M, near, far, W, H, rgb8([[200, 100, 50]]),
                       color_mode=osplat.COLOR_RGB8).reshape(3, H, W)
    sx, sy = centre64(M, p, W, H)
    for py in range(H):
        for px in range(W):
            d2 = (px + 0.5 - sx) ** 2 + (py + 0.5 - sy) ** 2
            a = alpha(d2) if d2 <= (3 * SIG) ** 2 else 0.0
            for c, v in enumerate((200, 100, 50)):
                assert img[c, py, px] == pytest.approx(v / 255 * a, abs=2e-6)
    assert img[:, int(sy), int(sx)].max() > 0.5


def test_two_gaussians_composite():
    """Front colour c1 with alpha a1 over back colour c2 with alpha a2:
    C = c1 a1 + c2 a2 (1 - a1), regardless of index order."""
    W, H = 16, 16
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    front = (0.02, 0.01, -1.0)
    back = (0.05, -0.03, -2.0)
    for order in ((front, back), (back, front)):
        xs, ys, zs = (np.array([q[k] for q in order], np.float32) for k in range(3))
        cols = [[255, 0, 0], [0, 0, 255]] if order[0] is front else [[0, 0, 255], [255, 0, 0]]
        img = osplat.splat(xs, ys, zs, M, near, far, W, H, rgb8(cols), color_mode=osplat.COLOR_RGB8).reshape(3, H, W)
        f = centre64(M, front, W, H)
        b = centre64(M, back, W, H)
        for py in range(H):
            for px in range(W):
                d1 = (px + 0.5 - f[0]) ** 2 + (py + 0.5 - f[1]) ** 2
                d2 = (px + 0.5 - b[0]) ** 2 + (py + 0.5 - b[1]) ** 2
                a1 = alpha(d1) if d1 <= 9 * SIG * SIG else 0.0
                a2 = alpha(d2) if d2 <= 9 * SIG * SIG else 0.0
                assert img[0, py, px] == pytest.approx(a1, abs=2e-6)
                assert img[2, py, px] == pytest.approx(a2 * (1 - a1), abs=2e-6)
                assert img[1, py, px] == 0.0


def test_early_termination():
    """Three coincident opaque layers: after two, T = 1e-4 * 0.99 ... the third
    would take T below 1e-4, so it is dropped."""
    W, H = 8, 8
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    # centre exactly on a pixel centre: sx = 4.5 -> x/w*0.5+0.5 = 4.5/8
    xw = (4.5 / 8 - 0.5) * 2
    xs = np.array([xw, xw, xw], np.float32)
    ys = np.array([-xw, -xw, -xw], np.float32)
    zs = np.array([-1.0, -2.0, -3.0], np.float32)
    xs2 = xs * np.array([1, 2, 3], np.float32)
    ys2 = ys * np.array([1, 2, 3], np.float32)
    img = osplat.splat(xs2, ys2, zs, M, near, far, W, H, rgb8([[255, 0, 0], [0, 255, 0], [0, 0, 255]]),
                       color_mode=osplat.COLOR_RGB8).reshape(3, H, W)
    p = img[:, 4, 4]
    assert p[0] == pytest.approx(0.99, abs=1e-6)
    assert p[1] == pytest.approx(0.99 * 0.01, abs=1e-6)
    assert p[2] == 0.0


def test_ties_blend_lower_index_first():
    W, H = 8, 8
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    xs = np.array([0.01, 0.01], np.float32)
    ys = np.array([0.02, 0.02], np.float32)
    zs = np.array([-1.5, -1.5], np.float32)
    img = osplat.splat(xs, ys, zs, M, near, far, W, H, rgb8([[255, 0, 0], [0, 255, 0]]),
                       color_mode=osplat.COLOR_RGB8)
    k = int(np.argmax(img[0]))
    assert img[0, k] > img[1, k] > 0


def test_footprint_is_three_sigma_and_culled_points_vanish():
    W, H = 40, 40
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    # one visible point, one behind the camera, one outside the image, one NaN
    xs = np.array([0.0, 0.0, 5.0, np.nan], np.float32)
    ys = np.array([0.0, 0.0, 0.0, 0.0], np.float32)
    zs = np.array([-1.0, 1.0, -1.0, -1.0], np.float32)
    img = osplat.splat(xs, ys, zs, M, near, far, W, H, rgb8([[255, 255, 255]] * 4),
                       color_mode=osplat.COLOR_RGB8).reshape(3, H, W)
    sx, sy = centre64(M, (0, 0, -1), W, H)
    yy, xx = np.mgrid[0:H, 0:W]
    d2 = (xx + 0.5 - sx) ** 2 + (yy + 0.5 - sy) ** 2
    assert (img[0][d2 > 9 * SIG * SIG + 1e-6] == 0).all()
    assert (img[0][d2 <= 9 * SIG * SIG - 1e-6] > 0).all()
    assert np.count_nonzero(img[0]) == np.count_nonzero(d2 <= 9 * SIG * SIG)


def test_lut_mode_matches_rgb_table():
    W, H = 16, 16
    M, near, far = ocam.clip_matrix(cam_identity(), W, H)
    lut = scenes.colour_lut()
    s = np.array([0.3], np.float32)
    img = osplat.splat(np.array([0.0], np.float32), np.array([0.0], np.float32), np.array([-1.0], np.float32),
                       M, near, far, W, H, [s], color_mode=osplat.COLOR_LUT, lut=lut, lut_attr=0,
                       lut_min=0.0, lut_inv_range=1.0).reshape(3, H, W)
    q = int(0.3 * 256)
    k = np.unravel_index(np.argmax(img[0]), (H, W))
    a = img[0][k] / lut[q, 0]
    np.testing.assert_allclose(img[:, k[0], k[1]], lut[q].astype(np.float64) * a, rtol=1e-6)


def test_permutation_invariance_distinct_depths():
    sc = scenes.unit_cube(n=3000, seed=21, W=64, H=48)
    cam = scenes.Camera(eye=(1.8, 1.6, 1.4), target=(0.5, 0.5, 0.5))
    M, near, far = ocam.clip_matrix(cam, sc.W, sc.H)
    lut = scenes.colour_lut()
    kw = dict(color_mode=osplat.COLOR_LUT, lut=lut, lut_attr=3, lut_min=0.0, lut_inv_range=1 / 3.5)
    a = osplat.splat(sc.x, sc.y, sc.z, M, near, far, sc.W, sc.H, sc.attrs, **kw)
    perm = np.random.default_rng(0).permutation(sc.n)
    b = osplat.splat(sc.x[perm], sc.y[perm], sc.z[perm], M, near, far, sc.W, sc.H, [t[perm] for t in sc.attrs], **kw)
    np.testing.assert_allclose(a, b, atol=1e-12)
    assert a.max() > 0.3


# ---------------------------------------------------------------------------
# anisotropic splat (Gaussians elongated along the velocity)
# ---------------------------------------------------------------------------

IDENT90 = scenes.Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fovy_deg=90.0)


def aniso_one(v, stretch, W=48, H=48, d=2.0, sigma=1.5):
    from oracle import splat as osplat
    M, near, far = ocam.clip_matrix(IDENT90, W, H)
    x = np.array([0.0], np.float32)
    y = np.array([0.0], np.float32)
    z = np.array([-d], np.float32)
    c = np.ones(1, np.float32)
    attrs = [np.array([v[0]], np.float32), np.array([v[1]], np.float32), np.array([v[2]], np.float32), c]
    lut = np.ones((256, 3), np.float32)
    return osplat.splat_aniso(x, y, z, M, near, far, W, H, attrs, vel_attr=0, stretch=stretch,
                              focal_px=ocam.focal_px(IDENT90, H), sigma=sigma, lut=lut, lut_attr=3)


def test_aniso_closed_form_on_axis():
    """On the optical axis of an identity view the screen covariance is
    sigma^2 diag(s, 1) for v along x (exactly, in real arithmetic): every
    pixel equals min(0.99, exp(-q/2)) with q = dx^2/(s sigma^2) + dy^2/sigma^2
    where q <= 9, and 0 elsewhere."""
    W = H = 48
    s, sig = 16.0, 1.5
    img = aniso_one((3.0, 0.0, 0.0), s, W, H, sigma=sig)[0].reshape(H, W)
    py, px = np.mgrid[0:H, 0:W]
    dx = px + 0.5 - W / 2
    dy = py + 0.5 - H / 2
    q = dx * dx / (s * sig * sig) + dy * dy / (sig * sig)
    want = np.where(q <= 9.0, np.minimum(0.99, np.exp(-q / 2)), 0.0)
    want = np.where(want >= 1 / 255, want, 0.0)
    edge = np.abs(q - 9.0) < 1e-3
    assert np.max(np.abs(img - want)[~edge]) < 1e-5
    assert (img > 0).sum() > 3 * (np.pi * 9 * sig * sig)   # about sqrt(s) = 4 times the round footprint


def test_aniso_reduces_to_round_without_stretch_or_velocity():
    from oracle import splat as osplat
    round_img = aniso_one((0.0, 0.0, 0.0), 300.0)          # no velocity: round
    ident = aniso_one((2.0, 1.0, 0.0), 1.0)                 # s = 1: round
    along_view = aniso_one((0.0, 0.0, 5.0), 300.0)          # v along the view axis: projects to nothing
    M, near, far = ocam.clip_matrix(IDENT90, 48, 48)
    iso = osplat.splat(np.zeros(1, np.float32), np.zeros(1, np.float32), np.array([-2.0], np.float32), M, near,
                       far, 48, 48, [np.ones(1, np.float32)], sigma=1.5, lut=np.ones((256, 3), np.float32),
                       lut_attr=0)
    for img in (round_img, ident, along_view):
        assert np.max(np.abs(img - iso)) < 1e-5


def test_aniso_orientation_follows_projected_velocity():
    # v along y (screen vertical): the footprint is tall; along x: wide
    tall = (aniso_one((0.0, 2.0, 0.0), 25.0)[0].reshape(48, 48) > 0)
    wide = (aniso_one((2.0, 0.0, 0.0), 25.0)[0].reshape(48, 48) > 0)
    assert tall.any(axis=1).sum() > 2 * tall.any(axis=0).sum()
    assert wide.any(axis=0).sum() > 2 * wide.any(axis=1).sum()
    assert np.array_equal(tall, wide.T)
