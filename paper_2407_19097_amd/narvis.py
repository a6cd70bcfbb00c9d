"""Python face of the C ABI: the same entry-point names, torch tensors in.

Each function converts tensors to device pointers and sizes, calls the
library on the current (or given) HIP stream and raises NarvisError on a
non-zero status.  No arithmetic of the method happens here.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import KEY_EMPTY, TILE_BOUNDS_MAX, NarvisError  # noqa: F401

RENDER_AUTO, RENDER_GLOBAL, RENDER_EARLYZ, RENDER_LDS = 0, 1, 2, 3

_DTYPE_CODE = None


def _dtype_code(t) -> int:
    global _DTYPE_CODE
    if _DTYPE_CODE is None:
        import torch
        _DTYPE_CODE = {torch.uint8: 0, torch.float16: 2, torch.float32: 3}
        if hasattr(torch, "uint16"):
            _DTYPE_CODE[torch.uint16] = 1
    try:
        return _DTYPE_CODE[t.dtype]
    except KeyError:
        raise TypeError(f"unsupported attribute dtype {t.dtype}") from None


def _stream_ptr(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


def camera_struct(cam) -> _lib.Camera:
    c = _lib.Camera()
    c.eye[:] = [float(v) for v in cam.eye]
    c.target[:] = [float(v) for v in cam.target]
    c.up[:] = [float(v) for v in cam.up]
    c.fovy_deg = float(cam.fovy_deg)
    c.znear = float(cam.znear)
    c.zfar = float(cam.zfar)
    return c


def points_struct(points) -> _lib.Points:
    x, y, z = points
    return _lib.Points(_ptr(x), _ptr(y), _ptr(z))


def attrs_struct(attrs: Sequence) -> _lib.Attrs:
    a = _lib.Attrs()
    a.count = len(attrs)
    if a.count > _lib.MAX_ATTRS:
        raise ValueError("at most 8 attribute streams")
    for k, t in enumerate(attrs):
        if t.dim() != 1:
            raise ValueError("attribute streams are 1-D tensors (strided views allowed)")
        a.a[k].data = t.data_ptr()
        a.a[k].dtype = _dtype_code(t)
        # a stride means nothing for a tensor of at most one element (torch may report 0)
        a.a[k].stride_bytes = (t.stride(0) if t.numel() > 1 else 1) * t.element_size()
    return a


@dataclass
class GBuffer:
    """Caller-owned output planes (torch tensors on the device)."""
    keys: object                  # int64 [H*W], bit pattern of the uint64 keys
    depth: object = None          # float32 [H*W]
    attr: object = None           # float32 [C][H*W]
    rgb: object = None            # float32 [3][H*W]
    vel2d: object = None          # float32 [4][H*W]
    lut: object = None            # float32 [256][3]
    lut_attr: int = -1
    lut_min: float = 0.0
    lut_inv_range: float = 1.0
    vel_attr: int = -1
    bounds: object = None         # uint8 [narvis_raster_bounds_bytes(W, H)] scratch of the bounded render
    hint: object = None           # int64 [H*W] keys of an earlier render (hinted bounded render)
    rgb_mode: int = 0             # COLOR_LUT or COLOR_RGB8 (three uint8 attributes from lut_attr)
    glyph: object = None          # uint8 [n] glyph mask (glyph-priority render), original point order
    radius: object = None         # float32 [H*W] projected splat radius in pixels
    radius_attr: int = -1         # attribute holding the world radius
    radius_focal_px: float = 0.0  # only read by narvis_raster_resolve (narvis_rasterize sets it)

    @staticmethod
    def allocate(W: int, H: int, nattr: int = 0, depth=True, rgb=False, vel2d=False, bounded=True, device="cuda"):
        import torch
        npx = W * H
        e = lambda *s: torch.empty(*s, device=device, dtype=torch.float32)
        return GBuffer(keys=torch.empty(npx, device=device, dtype=torch.int64),
                       depth=e(npx) if depth else None,
                       attr=e(nattr, npx) if nattr else None,
                       rgb=e(3, npx) if rgb else None,
                       vel2d=e(4, npx) if vel2d else None,
                       bounds=raster_bounds(W, H, device) if bounded else None)

    def struct(self) -> _lib.GBuffer:
        return _lib.GBuffer(_ptr(self.keys), _ptr(self.depth), _ptr(self.attr), _ptr(self.rgb), _ptr(self.vel2d),
                            _ptr(self.lut), int(self.lut_attr), float(self.lut_min), float(self.lut_inv_range),
                            int(self.vel_attr), _ptr(self.bounds),
                            0 if self.bounds is None else int(self.bounds.numel() * self.bounds.element_size()),
                            _ptr(self.hint), int(self.rgb_mode), _ptr(self.glyph), _ptr(self.radius),
                            int(self.radius_attr), float(self.radius_focal_px))


def narvis_status_string(status: int) -> str:
    return _lib.load().narvis_status_string(status).decode()


def narvis_camera_matrix(camera, W: int, H: int):
    """(float32[16] row-major clip matrix, near_f, far_f) composed on the host."""
    L = _lib.load()
    vp = (ctypes.c_float * 16)()
    nf, ff = ctypes.c_float(), ctypes.c_float()
    c = camera_struct(camera)
    _lib.check(L.narvis_camera_matrix(ctypes.byref(c), W, H, vp, ctypes.byref(nf), ctypes.byref(ff)),
               "narvis_camera_matrix")
    return np.frombuffer(vp, dtype=np.float32).copy(), np.float32(nf.value), np.float32(ff.value)


def narvis_camera_focal_px(camera, H: int) -> float:
    c = camera_struct(camera)
    f = ctypes.c_float()
    _lib.check(_lib.load().narvis_camera_focal_px(ctypes.byref(c), H, ctypes.byref(f)), "narvis_camera_focal_px")
    return float(f.value)


def _vp(vp) -> ctypes.Array:
    arr = np.ascontiguousarray(vp, dtype=np.float32).reshape(16)
    return (ctypes.c_float * 16)(*arr.tolist())


def narvis_raster_clear(keys, W: int, H: int, stream=None) -> None:
    _lib.check(_lib.load().narvis_raster_clear(_ptr(keys), W, H, _stream_ptr(stream)), "narvis_raster_clear")


def narvis_raster_bounds_bytes(W: int, H: int) -> int:
    return int(_lib.load().narvis_raster_bounds_bytes(W, H))


def raster_bounds(W: int, H: int, device="cuda"):
    """Scratch tensor for the bounded render of a W x H image."""
    import torch
    return torch.empty(narvis_raster_bounds_bytes(W, H), device=device, dtype=torch.uint8)


def narvis_raster_render(points, n: int, vp, near_f, far_f, W: int, H: int, keys, variant: int = RENDER_AUTO,
                         grid_blocks: int = 0, bounds=None, hint_keys=None, glyph=None, stream=None) -> None:
    p = points_struct(points)
    nb = 0 if bounds is None else int(bounds.numel() * bounds.element_size())
    o = _lib.RasterOpts(int(variant), int(grid_blocks), _ptr(bounds), nb, _ptr(hint_keys), _ptr(glyph))
    _lib.check(_lib.load().narvis_raster_render(ctypes.byref(p), int(n), _vp(vp), float(near_f), float(far_f), W, H,
                                                _ptr(keys), ctypes.byref(o), _stream_ptr(stream)),
               "narvis_raster_render")


def narvis_raster_resolve(points, attrs, n: int, vp, W: int, H: int, gbuf: GBuffer, stream=None) -> None:
    p = points_struct(points) if points is not None else _lib.Points()
    a = attrs_struct(attrs or [])
    g = gbuf.struct()
    _lib.check(_lib.load().narvis_raster_resolve(ctypes.byref(p), ctypes.byref(a), int(n), _vp(vp), W, H,
                                                 ctypes.byref(g), _stream_ptr(stream)), "narvis_raster_resolve")


def narvis_rasterize(points, attrs, n: int, camera, W: int, H: int, gbuf: GBuffer, stream=None) -> None:
    p = points_struct(points)
    a = attrs_struct(attrs or [])
    c = camera_struct(camera)
    g = gbuf.struct()
    _lib.check(_lib.load().narvis_rasterize(ctypes.byref(p), ctypes.byref(a), int(n), ctypes.byref(c), W, H,
                                            ctypes.byref(g), _stream_ptr(stream)), "narvis_rasterize")


def narvis_rasterize_static(points, attrs, n: int, camera, W: int, H: int, gbuf: GBuffer, stream=None) -> None:
    """Whole frame without any allocation: the bounds scratch is the library's
    static device array (gbuf.bounds must be None)."""
    p = points_struct(points)
    a = attrs_struct(attrs or [])
    c = camera_struct(camera)
    g = gbuf.struct()
    _lib.check(_lib.load().narvis_rasterize_static(ctypes.byref(p), ctypes.byref(a), int(n), ctypes.byref(c), W, H,
                                                   ctypes.byref(g), _stream_ptr(stream)), "narvis_rasterize_static")


STATIC_MAX_PIXELS = 3840 * 2160
LAYOUT_BATCH = 2048


class Layout:
    """Morton layout of a point cloud in caller-owned device tensors: x, y, z
    float32 [n] in layout order, index uint32 (as int32) [n] original index,
    boxes float32 [nbatch][8]; with sample=True also the render's depth
    sample (every 8th point: sx, sy, sz, sindex [ceil(n / 8)], sboxes)."""

    def __init__(self, n: int, device="cuda", sample: bool = True):
        import torch
        L = _lib.load()
        self.n = int(n)
        nb = int(L.narvis_layout_batches(self.n))
        e = lambda m: torch.empty(max(m, 4), dtype=torch.float32, device=device)
        self.x, self.y, self.z = e(self.n), e(self.n), e(self.n)
        self.index = torch.empty(max(self.n, 4), dtype=torch.int32, device=device)
        self.boxes = torch.empty((max(nb, 1), 8), dtype=torch.float32, device=device)
        self.sample = bool(sample)
        if self.sample:
            ns = int(L.narvis_layout_samples(self.n))
            nsb = int(L.narvis_layout_batches(ns))
            self.sx, self.sy, self.sz = e(ns), e(ns), e(ns)
            self.sindex = torch.empty(max(ns, 4), dtype=torch.int32, device=device)
            self.sboxes = torch.empty((max(nsb, 1), 8), dtype=torch.float32, device=device)

    def struct(self) -> _lib.Layout:
        if not self.sample:
            return _lib.Layout(_ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.index), _ptr(self.boxes))
        return _lib.Layout(_ptr(self.x), _ptr(self.y), _ptr(self.z), _ptr(self.index), _ptr(self.boxes),
                           _ptr(self.sx), _ptr(self.sy), _ptr(self.sz), _ptr(self.sindex), _ptr(self.sboxes))


def narvis_knn_radius_workspace_size(n: int) -> int:
    return int(_lib.load().narvis_knn_radius_workspace_size(int(n)))


def narvis_knn_radius(points, n: int, radius, workspace=None, stream=None):
    """World splat radius (mean distance to the four nearest neighbours) of
    every point into radius (float32 [n] device tensor).  Returns (cell edge,
    points settled by the full scan).  Synchronises the stream."""
    import torch
    p = points_struct(points)
    ws = workspace if workspace is not None else torch.empty(max(256, narvis_knn_radius_workspace_size(n)),
                                                              dtype=torch.uint8, device=radius.device)
    cell, unres = ctypes.c_float(), ctypes.c_uint32()
    _lib.check(_lib.load().narvis_knn_radius(ctypes.byref(p), int(n), _ptr(radius), _ptr(ws),
                                             ws.numel() * ws.element_size(), ctypes.byref(cell), ctypes.byref(unres),
                                             _stream_ptr(stream)), "narvis_knn_radius")
    return float(cell.value), int(unres.value)


def narvis_layout_workspace_size(n: int) -> int:
    return int(_lib.load().narvis_layout_workspace_size(int(n)))


def narvis_layout_build(points, n: int, layout: Layout, workspace, stream=None) -> None:
    p = points_struct(points)
    L = layout.struct()
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_layout_build(ctypes.byref(p), int(n), ctypes.byref(L), _ptr(workspace), nbytes,
                                               _stream_ptr(stream)), "narvis_layout_build")


def build_layout(points, n: int, device="cuda", sample: bool = True) -> Layout:
    """Allocate a Layout and build it (the workspace is freed afterwards)."""
    import torch
    L = Layout(n, device, sample=sample)
    ws = torch.empty(max(1, narvis_layout_workspace_size(n)), dtype=torch.uint8, device=device)
    narvis_layout_build(points, n, L, ws)
    del ws
    return L


def narvis_raster_render_layout(layout: Layout, n: int, vp, near_f, far_f, W: int, H: int, keys, grid_blocks: int = 0,
                                bounds=None, stream=None) -> None:
    L = layout.struct()
    nb = 0 if bounds is None else int(bounds.numel() * bounds.element_size())
    o = _lib.RasterOpts(RENDER_AUTO, int(grid_blocks), _ptr(bounds), nb, None, None)
    _lib.check(_lib.load().narvis_raster_render_layout(ctypes.byref(L), int(n), _vp(vp), float(near_f), float(far_f),
                                                       W, H, _ptr(keys), ctypes.byref(o), _stream_ptr(stream)),
               "narvis_raster_render_layout")


def narvis_rasterize_layout(layout: Layout, points, attrs, n: int, camera, W: int, H: int, gbuf: GBuffer,
                            stream=None) -> None:
    """points: the original-order coordinates (only read for vel2d; may be None otherwise)."""
    L = layout.struct()
    p = points_struct(points) if points is not None else _lib.Points()
    a = attrs_struct(attrs or [])
    c = camera_struct(camera)
    g = gbuf.struct()
    _lib.check(_lib.load().narvis_rasterize_layout(ctypes.byref(L), ctypes.byref(p), ctypes.byref(a), int(n),
                                                   ctypes.byref(c), W, H, ctypes.byref(g), _stream_ptr(stream)),
               "narvis_rasterize_layout")


COLOR_LUT, COLOR_RGB8 = 0, 1


@dataclass
class SplatParams:
    sigma_px: float = 1.5
    opacity: float = 1.0
    color_mode: int = COLOR_LUT
    color_attr: int = 0
    lut: object = None            # float32 [256][3] device tensor for COLOR_LUT
    lut_min: float = 0.0
    lut_inv_range: float = 1.0
    aniso: int = 0                # 1: Gaussians elongated along the velocity (attributes vel_attr..+2)
    vel_attr: int = -1
    stretch: float = 1.0          # s of S = diag(s, 1, 1)
    max_pairs: int = 0            # pair capacity; 0 = isotropic worst case (aniso: narvis_splat_count_pairs)

    def struct(self) -> _lib.SplatParams:
        return _lib.SplatParams(float(self.sigma_px), float(self.opacity), int(self.color_mode),
                                int(self.color_attr), _ptr(self.lut), float(self.lut_min), float(self.lut_inv_range),
                                int(self.aniso), int(self.vel_attr), float(self.stretch), 0.0, int(self.max_pairs))


def narvis_splat_workspace_size(n: int, W: int, H: int, params: SplatParams) -> int:
    p = params.struct()
    return int(_lib.load().narvis_splat_workspace_size(int(n), W, H, ctypes.byref(p)))


def narvis_splat(points, attrs, n: int, camera, W: int, H: int, img, params: SplatParams, workspace,
                 stream=None) -> None:
    """img: float32 [3][H*W] device tensor; workspace: uint8 device tensor of
    at least narvis_splat_workspace_size bytes."""
    pt = points_struct(points)
    a = attrs_struct(attrs or [])
    c = camera_struct(camera)
    p = params.struct()
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_splat(ctypes.byref(pt), ctypes.byref(a), int(n), ctypes.byref(c), W, H, _ptr(img),
                                        ctypes.byref(p), _ptr(workspace), nbytes, _stream_ptr(stream)),
               "narvis_splat")


def narvis_splat_count_pairs(points, attrs, n: int, camera, W: int, H: int, params: SplatParams, workspace,
                             stream=None) -> int:
    """Exact number of (tile, point) pairs narvis_splat emits (synchronises)."""
    pt = points_struct(points)
    a = attrs_struct(attrs or [])
    c = camera_struct(camera)
    p = params.struct()
    out = ctypes.c_uint64()
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_splat_count_pairs(ctypes.byref(pt), ctypes.byref(a), int(n), ctypes.byref(c), W, H,
                                                    ctypes.byref(p), _ptr(workspace), nbytes, ctypes.byref(out),
                                                    _stream_ptr(stream)), "narvis_splat_count_pairs")
    return int(out.value)


def narvis_splat_pair_count(workspace, n: int, W: int, H: int, params: SplatParams, stream=None) -> int:
    """(tile, key) pairs the last narvis_splat on `workspace` sorted (synchronises the stream)."""
    p = params.struct()
    out = ctypes.c_uint64()
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_splat_pair_count(_ptr(workspace), nbytes, int(n), W, H, ctypes.byref(p),
                                                   ctypes.byref(out), _stream_ptr(stream)), "narvis_splat_pair_count")
    return int(out.value)


PRECISION_BF16, PRECISION_FP8 = 0, 1


def narvis_net_param_count() -> int:
    return int(_lib.load().narvis_net_param_count())


class NetWeights:
    """Owner of a library parameter handle (narvis_weights_create / _destroy)."""

    def __init__(self, blob):
        blob = np.ascontiguousarray(blob, dtype=np.float32).reshape(-1)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().narvis_weights_create(blob.ctypes.data, blob.size, ctypes.byref(h)),
                   "narvis_weights_create")
        self.handle = h.value
        self.count = blob.size

    def read(self) -> np.ndarray:
        out = np.empty(self.count, dtype=np.float32)
        _lib.check(_lib.load().narvis_weights_read(self.handle, out.ctypes.data, self.count), "narvis_weights_read")
        return out

    def close(self):
        if self.handle:
            _lib.load().narvis_weights_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def narvis_postprocess_workspace_size(B: int, W: int, H: int) -> int:
    return int(_lib.load().narvis_postprocess_workspace_size(B, W, H))


def narvis_postprocess(weights: NetWeights, feat, B: int, W: int, H: int, img, workspace,
                       precision: int = PRECISION_BF16, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_postprocess(weights.handle, _ptr(feat), B, W, H, _ptr(img), precision,
                                              _ptr(workspace), nbytes, _stream_ptr(stream)), "narvis_postprocess")


def narvis_train_workspace_size(B: int, W: int, H: int) -> int:
    return int(_lib.load().narvis_train_workspace_size(B, W, H))


def narvis_train_step(weights: NetWeights, feat, target, B: int, W: int, H: int, lr: float, lam_tv: float,
                      loss_out, workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_train_step(weights.handle, _ptr(feat), _ptr(target), B, W, H, float(lr),
                                             float(lam_tv), _ptr(loss_out), _ptr(workspace), nbytes,
                                             _stream_ptr(stream)), "narvis_train_step")


def narvis_train_gradients(weights: NetWeights, feat, target, B: int, W: int, H: int, lam_tv: float, grad_out,
                           loss_out, workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_train_gradients(weights.handle, _ptr(feat), _ptr(target), B, W, H, float(lam_tv),
                                                  _ptr(grad_out), _ptr(loss_out), _ptr(workspace), nbytes,
                                                  _stream_ptr(stream)), "narvis_train_gradients")


def narvis_weights_calibrate_fp8(weights: NetWeights, feat, B: int, W: int, H: int, workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_weights_calibrate_fp8(weights.handle, _ptr(feat), B, W, H, _ptr(workspace), nbytes,
                                                        _stream_ptr(stream)), "narvis_weights_calibrate_fp8")


def narvis_weights_fp8_layers(weights: NetWeights) -> int:
    """Bit mask of the layers the last FP8 calibration put in FP8 (blob order)."""
    m = ctypes.c_uint32()
    _lib.check(_lib.load().narvis_weights_fp8_layers(weights.handle, ctypes.byref(m)), "narvis_weights_fp8_layers")
    return int(m.value)


def narvis_train_tensor(B: int, W: int, H: int, name: str):
    """(byte offset, channels, height, width, dtype) of a named tensor in the
    training workspace; dtype 0 = bfloat16 NHWC, 1 = fp32 planar."""
    off, c, h, w, dt = ctypes.c_size_t(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().narvis_train_tensor(B, W, H, name.encode(), ctypes.byref(off), ctypes.byref(c),
                                               ctypes.byref(h), ctypes.byref(w), ctypes.byref(dt)),
               "narvis_train_tensor")
    return int(off.value), int(c.value), int(h.value), int(w.value), int(dt.value)


# ---------------------------------------------------------------------------
# the paper's gated U-Net
# ---------------------------------------------------------------------------

UNET_WIDTHS = (64, 128, 256, 512, 1024)


def _widths(widths):
    return (ctypes.c_int32 * 5)(*[int(v) for v in widths])


def narvis_unet_param_count(widths=UNET_WIDTHS) -> int:
    return int(_lib.load().narvis_unet_param_count(_widths(widths)))


class UNet:
    """Library-owned parameters of the gated U-Net (create / destroy pair)."""

    def __init__(self, blob, widths=UNET_WIDTHS):
        blob = np.ascontiguousarray(blob, dtype=np.float32)
        self.widths = tuple(int(v) for v in widths)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().narvis_unet_create(_widths(self.widths), blob.ctypes.data, blob.size, ctypes.byref(h)),
                   "narvis_unet_create")
        self.handle = h
        self.count = blob.size

    def read(self) -> np.ndarray:
        out = np.empty(self.count, np.float32)
        _lib.check(_lib.load().narvis_unet_read(self.handle, out.ctypes.data, out.size), "narvis_unet_read")
        return out

    def close(self):
        if getattr(self, "handle", None):
            _lib.load().narvis_unet_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def narvis_unet_workspace_size(u: UNet, B: int, W: int, H: int, train: bool = False) -> int:
    return int(_lib.load().narvis_unet_workspace_size(u.handle, B, W, H, int(bool(train))))


def narvis_unet_forward(u: UNet, feat, B: int, W: int, H: int, img, workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_unet_forward(u.handle, _ptr(feat), B, W, H, _ptr(img), _ptr(workspace), nbytes,
                                               _stream_ptr(stream)), "narvis_unet_forward")


def narvis_unet_train_step(u: UNet, feat, target, B: int, W: int, H: int, lr: float, lam_tv: float, loss_out,
                           workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_unet_train_step(u.handle, _ptr(feat), _ptr(target), B, W, H, float(lr),
                                                  float(lam_tv), _ptr(loss_out), _ptr(workspace), nbytes,
                                                  _stream_ptr(stream)), "narvis_unet_train_step")


def narvis_unet_gradients(u: UNet, feat, target, B: int, W: int, H: int, lam_tv: float, grad_out, loss_out,
                          workspace, stream=None) -> None:
    nbytes = workspace.numel() * workspace.element_size()
    _lib.check(_lib.load().narvis_unet_gradients(u.handle, _ptr(feat), _ptr(target), B, W, H, float(lam_tv),
                                                 _ptr(grad_out), _ptr(loss_out), _ptr(workspace), nbytes,
                                                 _stream_ptr(stream)), "narvis_unet_gradients")
