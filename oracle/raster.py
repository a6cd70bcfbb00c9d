"""ctypes wrapper around the C raster oracle -- TEST INFRASTRUCTURE ONLY."""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
_lib = None


class _Attr(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("stride_bytes", ctypes.c_int32)]


_DT = {np.dtype(np.uint8): 0, np.dtype(np.uint16): 1, np.dtype(np.float16): 2, np.dtype(np.float32): 3}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        L.oracle_render.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_float, ctypes.c_float,
                                    ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_render_range.argtypes = [P, P, P, ctypes.c_uint64, ctypes.c_uint64, P, ctypes.c_float,
                                          ctypes.c_float, ctypes.c_int32, ctypes.c_int32, P]
        L.oracle_render_mt.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_int32, ctypes.c_int32, P, ctypes.c_int]
        L.oracle_render_mt.restype = ctypes.c_int
        L.oracle_render_glyph.argtypes = [P, P, P, ctypes.c_uint64, P, ctypes.c_float, ctypes.c_float,
                                          ctypes.c_int32, ctypes.c_int32, P, P]
        L.oracle_resolve_radius.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, ctypes.c_float, P]
        L.oracle_project_point.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                           ctypes.POINTER(ctypes.c_float)]
        L.oracle_project_point.restype = ctypes.c_int64
        L.oracle_resolve.argtypes = [P, ctypes.c_int32, ctypes.c_int32, P, P, P, P, P, ctypes.c_int32,
                                     P, P, P, P, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                     P, ctypes.c_int32, ctypes.c_int32]
        _lib = L
    return _lib


def _f32(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data


def render(x, y, z, M, near, far, W, H):
    """Key buffer uint64[H*W] of the render stage."""
    x, px = _f32(x)
    y, py = _f32(y)
    z, pz = _f32(z)
    M, pm = _f32(M)
    keys = np.empty(W * H, dtype=np.uint64)
    lib().oracle_render(px, py, pz, x.shape[0], pm, float(near), float(far), W, H, keys.ctypes.data)
    return keys


def render_glyph(x, y, z, M, near, far, W, H, glyph):
    """Key buffer of the glyph-priority render (glyph: uint8 [n], nonzero = glyph point)."""
    x, px = _f32(x)
    y, py = _f32(y)
    z, pz = _f32(z)
    M, pm = _f32(M)
    g = np.ascontiguousarray(glyph, dtype=np.uint8)
    keys = np.empty(W * H, dtype=np.uint64)
    lib().oracle_render_glyph(px, py, pz, x.shape[0], pm, float(near), float(far), W, H, g.ctypes.data,
                              keys.ctypes.data)
    return keys


def resolve_radius(keys, W, H, r_world, focal_px):
    """Projected splat radius plane [H*W] of a key buffer."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    r = np.ascontiguousarray(r_world, dtype=np.float32)
    out = np.empty(W * H, np.float32)
    lib().oracle_resolve_radius(keys.ctypes.data, W, H, r.ctypes.data, float(np.float32(focal_px)), out.ctypes.data)
    return out


def render_mt(x, y, z, M, near, far, W, H, threads):
    """render() on `threads` host threads (private key buffers merged by
    elementwise minimum: the same keys)."""
    x, px = _f32(x)
    y, py = _f32(y)
    z, pz = _f32(z)
    M, pm = _f32(M)
    keys = np.empty(W * H, dtype=np.uint64)
    if lib().oracle_render_mt(px, py, pz, x.shape[0], pm, float(near), float(far), W, H, keys.ctypes.data,
                              int(threads)) != 0:
        raise MemoryError("oracle_render_mt: no memory or threads")
    return keys


def render_range(x, y, z, i0, i1, M, near, far, W, H, keys):
    """Merge points [i0, i1) into ``keys`` (caller-initialised)."""
    M, pm = _f32(M)
    lib().oracle_render_range(x.ctypes.data, y.ctypes.data, z.ctypes.data, i0, i1, pm,
                              float(near), float(far), W, H, keys.ctypes.data)
    return keys


def project_point(M, near, far, W, H, x, y, z):
    M, pm = _f32(M)
    w = ctypes.c_float(0.0)
    p = lib().oracle_project_point(pm, float(near), float(far), W, H, float(np.float32(x)),
                                   float(np.float32(y)), float(np.float32(z)), ctypes.byref(w))
    return int(p), np.float32(w.value)


def _attr_array(attrs):
    arr = (_Attr * max(1, len(attrs)))()
    keep = []
    for k, a in enumerate(attrs):
        a = np.asarray(a)
        if a.ndim != 1:
            raise ValueError("attributes are 1-D arrays")
        keep.append(a)
        arr[k].data = a.ctypes.data
        arr[k].dtype = _DT[a.dtype]
        arr[k].stride_bytes = a.strides[0]
    return arr, keep


def resolve(keys, W, H, x, y, z, M, attrs, want_depth=True, want_attrs=True,
            lut=None, lut_attr=-1, lut_min=0.0, lut_inv_range=1.0, vel_attr=-1, rgb_mode=0):
    """Returns dict with depth [H*W], attrs [C][H*W], rgb [3][H*W], vel2d [4][H*W] as requested
    (rgb: lut given, or rgb_mode 1 = three uint8 attributes from lut_attr, scaled by 1/255)."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64)
    x, px = _f32(x)
    y, py = _f32(y)
    z, pz = _f32(z)
    M, pm = _f32(M)
    npx = W * H
    arr, keep = _attr_array(attrs)
    out = {}
    depth = np.empty(npx, np.float32) if want_depth else None
    chan = np.empty((len(attrs), npx), np.float32) if (want_attrs and attrs) else None
    rgb = np.empty((3, npx), np.float32) if (lut is not None or rgb_mode == 1) else None
    vel = np.empty((4, npx), np.float32) if vel_attr >= 0 else None
    lutc = np.ascontiguousarray(lut, dtype=np.float32).reshape(-1) if lut is not None else None
    ptr = lambda a: None if a is None else a.ctypes.data
    lib().oracle_resolve(keys.ctypes.data, W, H, px, py, pz, pm, ctypes.cast(arr, ctypes.c_void_p),
                         len(attrs), ptr(depth), ptr(chan), ptr(rgb), ptr(lutc), lut_attr,
                         float(lut_min), float(lut_inv_range), ptr(vel), vel_attr, int(rgb_mode))
    if depth is not None:
        out["depth"] = depth
    if chan is not None:
        out["attrs"] = chan
    if rgb is not None:
        out["rgb"] = rgb
    if vel is not None:
        out["vel2d"] = vel
    del keep
    return out
