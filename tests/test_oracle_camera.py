"""Pins for the oracle's FP64 camera composition (Sec. 3.3 camera: vertical
field of view 60 degrees, near 0.1, far 2e5)."""
import math

import numpy as np
import pytest

from oracle import camera as ocam
from paper_2407_19097_amd import scenes


def test_identity_view_gives_projection():
    cam = scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0))
    V = ocam.look_at(cam.eye, cam.target, cam.up)
    np.testing.assert_array_equal(V, np.eye(4))
    M64 = ocam.clip_matrix64(cam, 1920, 1080)
    t = math.tan(math.radians(30.0))
    assert M64[0, 0] == pytest.approx(1.0 / (t * 1920 / 1080), rel=1e-15)
    assert M64[1, 1] == pytest.approx(1.0 / t, rel=1e-15)
    np.testing.assert_array_equal(M64[3], [0, 0, -1, 0])


@pytest.mark.parametrize("seed", range(5))
def test_axis_point_and_depth(seed):
    """A point eye + d*f projects to the image centre with w = d; a point one
    unit up lands above the centre, one unit right to the right of it."""
    rng = np.random.default_rng(seed)
    eye = rng.normal(size=3) * 3
    target = rng.normal(size=3)
    cam = scenes.Camera(eye=tuple(eye), target=tuple(target))
    W, H = 800, 600
    M = ocam.clip_matrix64(cam, W, H)
    f = (target - eye) / np.linalg.norm(target - eye)
    for d in (0.3, 2.0, 50.0):
        c = M @ np.append(eye + d * f, 1.0)
        assert c[3] == pytest.approx(d, rel=1e-12)
        assert abs(c[0] / c[3]) < 1e-12 and abs(c[1] / c[3]) < 1e-12
    up = np.array([0, 0, 1.0])
    upv = up - (up @ f) * f
    upv /= np.linalg.norm(upv)
    right = np.cross(f, upv)
    c = M @ np.append(eye + 2 * f + 0.1 * upv, 1.0)
    assert c[1] > 0 and abs(c[0]) < 1e-9
    c = M @ np.append(eye + 2 * f + 0.1 * right, 1.0)
    assert c[0] > 0 and abs(c[1]) < 1e-9
    # field of view: a point at the top edge of the frustum has ndc y = 1
    c = M @ np.append(eye + 2 * f + 2 * math.tan(math.radians(30)) * upv, 1.0)
    assert c[1] / c[3] == pytest.approx(1.0, rel=1e-12)


def test_degenerate_cameras_rejected():
    with pytest.raises(ValueError):
        ocam.look_at((0, 0, 0), (0, 0, 0), (0, 0, 1))
    with pytest.raises(ValueError):
        ocam.look_at((0, 0, 0), (0, 0, 5), (0, 0, 1))
    with pytest.raises(ValueError):
        ocam.perspective(0.0, 1.0, 0.1, 10)
    with pytest.raises(ValueError):
        ocam.perspective(60.0, 1.0, 1.0, 0.5)
