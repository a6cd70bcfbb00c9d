"""FP64 camera composition for the oracle -- TEST INFRASTRUCTURE ONLY.

Parity unpinned by the paper: Sec. 3.3 fixes only the training camera (vertical
field of view 60 degrees, near 0.1, far 2e5).  The reading used here is the
standard right-handed look-at view matrix V and the OpenGL perspective matrix
P with aspect W/H; the clip-space transform is M = P V composed in float64 as a
full 4x4 product and rounded once per entry to float32.  Row 3 of M is the
view-axis distance, which is the depth the rasterizer stores.
"""
from __future__ import annotations

import math

import numpy as np


def look_at(eye, target, up) -> np.ndarray:
    eye = np.asarray(eye, dtype=np.float64)
    target = np.asarray(target, dtype=np.float64)
    up = np.asarray(up, dtype=np.float64)
    f = target - eye
    fn = math.sqrt(float(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]))
    if not fn > 0.0:
        raise ValueError("eye and target coincide")
    f = f / fn
    s = np.cross(f, up)
    sn = math.sqrt(float(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]))
    if not sn > 1e-12:
        raise ValueError("up is parallel to the viewing direction")
    s = s / sn
    u = np.cross(s, f)
    V = np.eye(4, dtype=np.float64)
    V[0, :3], V[1, :3], V[2, :3] = s, u, -f
    V[0, 3] = -float(s @ eye)
    V[1, 3] = -float(u @ eye)
    V[2, 3] = float(f @ eye)
    return V


def perspective(fovy_deg, aspect, znear, zfar) -> np.ndarray:
    if not (0.0 < fovy_deg < 180.0) or not (0.0 < znear < zfar):
        raise ValueError("bad projection parameters")
    t = math.tan(math.radians(fovy_deg) / 2.0)
    P = np.zeros((4, 4), dtype=np.float64)
    P[0, 0] = 1.0 / (aspect * t)
    P[1, 1] = 1.0 / t
    P[2, 2] = -(zfar + znear) / (zfar - znear)
    P[2, 3] = -2.0 * zfar * znear / (zfar - znear)
    P[3, 2] = -1.0
    return P


def clip_matrix64(cam, W: int, H: int) -> np.ndarray:
    """M = P V in float64 for a camera with eye/target/up/fovy_deg/znear/zfar."""
    return perspective(cam.fovy_deg, W / H, cam.znear, cam.zfar) @ look_at(cam.eye, cam.target, cam.up)


def clip_matrix(cam, W: int, H: int):
    """(M as float32 row-major [16], near as float32, far as float32)."""
    M = clip_matrix64(cam, W, H).astype(np.float32).reshape(16)
    return M, np.float32(cam.znear), np.float32(cam.zfar)


def focal_px(cam, H: int) -> np.float32:
    """Focal length in pixels for an image H pixels high, (H / 2) / tan(fovy / 2),
    in float64 rounded once to float32 (the scale of the projected splat radius)."""
    return np.float32(H * 0.5 / math.tan(math.radians(cam.fovy_deg) / 2.0))
