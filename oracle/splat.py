"""ctypes wrapper around the C splat oracle -- TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes

import numpy as np

from . import raster as _r

COLOR_LUT, COLOR_RGB8 = 0, 1
_bound = False


def _lib():
    global _bound
    L = _r.lib()
    if not _bound:
        P = ctypes.c_void_p
        L.oracle_splat.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_int32, P, ctypes.c_int32,
                                   P, ctypes.c_int32, ctypes.c_float, ctypes.c_float, P, P]
        L.oracle_splat.restype = ctypes.c_int
        L.oracle_splat_aniso.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_float, ctypes.c_float, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_int32, P,
                                         ctypes.c_int32, P, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                         ctypes.c_int32, ctypes.c_float, ctypes.c_float, P, P, P]
        L.oracle_splat_aniso.restype = ctypes.c_int
        _bound = True
    return L


def splat(x, y, z, M, near, far, W, H, attrs, sigma=1.5, opacity=1.0, color_mode=COLOR_LUT,
          lut=None, lut_attr=0, lut_min=0.0, lut_inv_range=1.0, with_fragile=False):
    """float64 image [3][H*W] of the isotropic front-to-back Gaussian splat
    (and, with with_fragile, the uint8 [H*W] near-threshold flags)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    M = np.ascontiguousarray(M, np.float32).reshape(16)
    arr, keep = _r._attr_array(attrs)
    lutc = np.ascontiguousarray(lut if lut is not None else np.zeros((256, 3)), np.float32).reshape(-1)
    img = np.empty((3, W * H), np.float64)
    frag = np.empty(W * H, np.uint8) if with_fragile else None
    rc = _lib().oracle_splat(x.ctypes.data, y.ctypes.data, z.ctypes.data, x.shape[0], M.ctypes.data, float(near),
                             float(far), W, H, float(sigma), float(opacity), color_mode,
                             ctypes.cast(arr, ctypes.c_void_p), len(attrs), lutc.ctypes.data, lut_attr,
                             float(lut_min), float(lut_inv_range), img.ctypes.data,
                             None if frag is None else frag.ctypes.data)
    del keep
    if rc != 0:
        raise MemoryError("oracle_splat could not allocate")
    return (img, frag) if with_fragile else img


def splat_aniso(x, y, z, M, near, far, W, H, attrs, vel_attr, stretch, focal_px, sigma=1.5, opacity=1.0,
                color_mode=COLOR_LUT, lut=None, lut_attr=0, lut_min=0.0, lut_inv_range=1.0, window=None,
                with_fragile=False):
    """float64 image [3][H*W] of the splat elongated along the velocity
    (attributes vel_attr..vel_attr+2); window = (x0, y0, x1, y1) composites
    only those pixels (the rest stay 0)."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.ascontiguousarray(y, np.float32)
    z = np.ascontiguousarray(z, np.float32)
    M = np.ascontiguousarray(M, np.float32).reshape(16)
    arr, keep = _r._attr_array(attrs)
    lutc = np.ascontiguousarray(lut if lut is not None else np.zeros((256, 3)), np.float32).reshape(-1)
    win = None if window is None else np.ascontiguousarray(window, np.int32)
    img = np.empty((3, W * H), np.float64)
    frag = np.empty(W * H, np.uint8) if with_fragile else None
    rc = _lib().oracle_splat_aniso(x.ctypes.data, y.ctypes.data, z.ctypes.data, x.shape[0], M.ctypes.data,
                                   float(near), float(far), W, H, float(sigma), float(opacity), color_mode,
                                   ctypes.cast(arr, ctypes.c_void_p), len(attrs), lutc.ctypes.data, lut_attr,
                                   float(lut_min), float(lut_inv_range), int(vel_attr), float(stretch),
                                   float(np.float32(focal_px)), None if win is None else win.ctypes.data,
                                   img.ctypes.data, None if frag is None else frag.ctypes.data)
    del keep
    if rc != 0:
        raise MemoryError("oracle_splat_aniso could not allocate")
    return (img, frag) if with_fragile else img
