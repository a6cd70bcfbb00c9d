"""ctypes binding of libnarvis.so: structure layouts and symbol signatures.

Argument marshalling only.  The library is loaded from this package's
directory; if it has not been built the import of any entry point fails with
an error that says so -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnarvis.so")

MAX_ATTRS = 8
KEY_EMPTY = 0xFFFFFFFFFFFFFFFF
TILE_BOUNDS_MAX = 8192

STATUS = {0: "NARVIS_OK", -1: "NARVIS_ERR_INVALID_ARG", -2: "NARVIS_ERR_OUT_OF_MEMORY",
          -3: "NARVIS_ERR_DEVICE", -4: "NARVIS_ERR_UNSUPPORTED", -5: "NARVIS_ERR_WORKSPACE"}


class NarvisError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}")


class Points(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p)]


class Attr(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("stride_bytes", ctypes.c_int32)]


class Attrs(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32), ("a", Attr * MAX_ATTRS)]


class Camera(ctypes.Structure):
    _fields_ = [("eye", ctypes.c_double * 3), ("target", ctypes.c_double * 3), ("up", ctypes.c_double * 3),
                ("fovy_deg", ctypes.c_double), ("znear", ctypes.c_double), ("zfar", ctypes.c_double)]


class GBuffer(ctypes.Structure):
    _fields_ = [("keys", ctypes.c_void_p), ("depth", ctypes.c_void_p), ("attr", ctypes.c_void_p),
                ("rgb", ctypes.c_void_p), ("vel2d", ctypes.c_void_p), ("lut", ctypes.c_void_p),
                ("lut_attr", ctypes.c_int32), ("lut_min", ctypes.c_float), ("lut_inv_range", ctypes.c_float),
                ("vel_attr", ctypes.c_int32), ("bounds", ctypes.c_void_p), ("bounds_bytes", ctypes.c_size_t),
                ("hint_keys", ctypes.c_void_p), ("rgb_mode", ctypes.c_int32), ("glyph", ctypes.c_void_p),
                ("radius", ctypes.c_void_p), ("radius_attr", ctypes.c_int32), ("radius_focal_px", ctypes.c_float)]


class RasterOpts(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("grid_blocks", ctypes.c_int32), ("bounds", ctypes.c_void_p),
                ("bounds_bytes", ctypes.c_size_t), ("hint_keys", ctypes.c_void_p), ("glyph", ctypes.c_void_p)]


class SplatParams(ctypes.Structure):
    _fields_ = [("sigma_px", ctypes.c_float), ("opacity", ctypes.c_float), ("color_mode", ctypes.c_int32),
                ("color_attr", ctypes.c_int32), ("lut", ctypes.c_void_p), ("lut_min", ctypes.c_float),
                ("lut_inv_range", ctypes.c_float), ("aniso", ctypes.c_int32), ("vel_attr", ctypes.c_int32),
                ("stretch", ctypes.c_float), ("focal_px", ctypes.c_float), ("max_pairs", ctypes.c_uint64)]


class Layout(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("z", ctypes.c_void_p), ("index", ctypes.c_void_p),
                ("boxes", ctypes.c_void_p), ("sx", ctypes.c_void_p), ("sy", ctypes.c_void_p), ("sz", ctypes.c_void_p),
                ("sindex", ctypes.c_void_p), ("sboxes", ctypes.c_void_p)]


_P = ctypes.c_void_p
_F16 = ctypes.c_float * 16

# name -> (restype, argtypes); every entry point of include/narvis.h
SIGNATURES = {
    "narvis_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "narvis_camera_matrix": (ctypes.c_int, [ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32, _F16,
                                            ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "narvis_camera_focal_px": (ctypes.c_int, [ctypes.POINTER(Camera), ctypes.c_int32, ctypes.POINTER(ctypes.c_float)]),
    "narvis_raster_clear": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32, _P]),
    "narvis_raster_bounds_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32]),
    "narvis_raster_render": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.c_uint64, _F16, ctypes.c_float,
                                            ctypes.c_float, ctypes.c_int32, ctypes.c_int32, _P,
                                            ctypes.POINTER(RasterOpts), _P]),
    "narvis_raster_resolve": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.POINTER(Attrs), ctypes.c_uint64, _F16,
                                             ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(GBuffer), _P]),
    "narvis_rasterize": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.POINTER(Attrs), ctypes.c_uint64,
                                        ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32,
                                        ctypes.POINTER(GBuffer), _P]),
    "narvis_knn_radius_workspace_size": (ctypes.c_size_t, [ctypes.c_uint64]),
    "narvis_knn_radius": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.c_uint64, _P, _P, ctypes.c_size_t,
                                         ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_uint32), _P]),
    "narvis_rasterize_static": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.POINTER(Attrs), ctypes.c_uint64,
                                               ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(GBuffer), _P]),
    "narvis_layout_batches": (ctypes.c_uint64, [ctypes.c_uint64]),
    "narvis_layout_samples": (ctypes.c_uint64, [ctypes.c_uint64]),
    "narvis_layout_workspace_size": (ctypes.c_size_t, [ctypes.c_uint64]),
    "narvis_layout_build": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.c_uint64, ctypes.POINTER(Layout), _P,
                                           ctypes.c_size_t, _P]),
    "narvis_raster_render_layout": (ctypes.c_int, [ctypes.POINTER(Layout), ctypes.c_uint64, _F16, ctypes.c_float,
                                                   ctypes.c_float, ctypes.c_int32, ctypes.c_int32, _P,
                                                   ctypes.POINTER(RasterOpts), _P]),
    "narvis_rasterize_layout": (ctypes.c_int, [ctypes.POINTER(Layout), ctypes.POINTER(Points), ctypes.POINTER(Attrs),
                                               ctypes.c_uint64, ctypes.POINTER(Camera), ctypes.c_int32,
                                               ctypes.c_int32, ctypes.POINTER(GBuffer), _P]),
    "narvis_splat_workspace_size": (ctypes.c_size_t, [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                                       ctypes.POINTER(SplatParams)]),
    "narvis_splat": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.POINTER(Attrs), ctypes.c_uint64,
                                    ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32, _P,
                                    ctypes.POINTER(SplatParams), _P, ctypes.c_size_t, _P]),
    "narvis_splat_count_pairs": (ctypes.c_int, [ctypes.POINTER(Points), ctypes.POINTER(Attrs), ctypes.c_uint64,
                                                ctypes.POINTER(Camera), ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(SplatParams), _P, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_uint64), _P]),
    "narvis_splat_pair_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.POINTER(SplatParams),
                                                ctypes.POINTER(ctypes.c_uint64), ctypes.c_void_p]),
    "narvis_net_param_count": (ctypes.c_size_t, []),
    "narvis_weights_create": (ctypes.c_int, [_P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_void_p)]),
    "narvis_weights_destroy": (None, [_P]),
    "narvis_weights_read": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "narvis_postprocess_workspace_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "narvis_postprocess": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                          ctypes.c_int32, _P, ctypes.c_size_t, _P]),
    "narvis_weights_calibrate_fp8": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P,
                                                    ctypes.c_size_t, _P]),
    "narvis_weights_fp8_layers": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_uint32)]),
    "narvis_unet_param_count": (ctypes.c_size_t, [ctypes.POINTER(ctypes.c_int32)]),
    "narvis_unet_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int32), _P, ctypes.c_size_t,
                                          ctypes.POINTER(ctypes.c_void_p)]),
    "narvis_unet_destroy": (None, [_P]),
    "narvis_unet_read": (ctypes.c_int, [_P, _P, ctypes.c_size_t]),
    "narvis_unet_workspace_size": (ctypes.c_size_t, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                     ctypes.c_int32]),
    "narvis_unet_forward": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                           ctypes.c_size_t, _P]),
    "narvis_unet_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, ctypes.c_float, _P, _P, ctypes.c_size_t, _P]),
    "narvis_unet_gradients": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                             ctypes.c_float, _P, _P, _P, ctypes.c_size_t, _P]),
    "narvis_train_workspace_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "narvis_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_float, ctypes.c_float, _P, _P, ctypes.c_size_t, _P]),
    "narvis_train_gradients": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_float, _P, _P, _P, ctypes.c_size_t, _P]),
    "narvis_train_tensor": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_char_p,
                                           ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load():
    """Load libnarvis.so (built by paper_2407_19097_amd.build) and bind every symbol."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run paper_2407_19097_amd/build.py "
                              "(the HIP library is the only implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str) -> None:
    if status != 0:
        raise NarvisError(status, where)
