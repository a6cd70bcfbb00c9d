"""The allocation-free whole-frame call (narvis_rasterize_static) against the
whole-frame call with a caller-owned bounds scratch (narvis_rasterize), bit
for bit on keys and every G-buffer plane, on two calls in a row, the second
with fewer points and a smaller image (the static scratch keeps the first
call's contents), then its argument checks (host-side rejections, nothing is
launched)."""
import ctypes

import numpy as np
import pytest

from paper_2407_19097_amd import _lib, narvis, scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def frame(sc, W, H, static):
    """Keys, depth, attribute, rgb and Vel2D planes of one whole-frame call."""
    d = torch.device("cuda")
    X, Y, Z = (torch.from_numpy(a).to(d) for a in (sc.x, sc.y, sc.z))
    A = [torch.from_numpy(a).to(d) for a in sc.attrs]
    g = narvis.GBuffer.allocate(W, H, nattr=len(A), depth=True, rgb=True, vel2d=True, bounded=not static)
    g.lut = torch.from_numpy(scenes.colour_lut()).to(d)
    g.lut_attr, g.lut_min, g.lut_inv_range = 3, 0.0, float(np.float32(1.0 / 3.0))
    g.vel_attr = 0
    # the planes start as garbage: the call must write every element
    for t in (g.depth, g.attr, g.rgb, g.vel2d):
        t.fill_(float("nan"))
    g.keys.fill_(7)
    if static:
        narvis.narvis_rasterize_static((X, Y, Z), A, sc.n, sc.cameras[0], W, H, g)
    else:
        narvis.narvis_rasterize((X, Y, Z), A, sc.n, sc.cameras[0], W, H, g)
    torch.cuda.synchronize()
    return {k: getattr(g, k).cpu().numpy().view(np.uint32 if k != "keys" else np.uint64)
            for k in ("keys", "depth", "attr", "rgb", "vel2d")}


@pytest.mark.parametrize("n,W,H", [(1_000_003, 1280, 720), (200_001, 512, 384)])
def test_static_scratch_matches_caller_scratch(n, W, H):
    print(f"\n[case] narvis_rasterize_static vs narvis_rasterize, unit cube n={n} at {W}x{H}", flush=True)
    sc = scenes.unit_cube(n=n, seed=11, W=W, H=H)
    assert n >= 4096 and W * H <= narvis.STATIC_MAX_PIXELS  # the bounded render applies
    want = frame(sc, W, H, static=False)
    got = frame(sc, W, H, static=True)
    covered = int((want["keys"] != np.uint64(0xFFFFFFFFFFFFFFFF)).sum())
    print(f"  {covered} covered pixels", flush=True)
    assert covered > 0
    for k in want:
        assert np.array_equal(got[k], want[k]), k


def test_static_rejects_what_does_not_fit():
    print("\n[case] narvis_rasterize_static argument checks (host side only)", flush=True)
    sc = scenes.unit_cube(n=4096, seed=3, W=64, H=64)
    d = torch.device("cuda")
    X, Y, Z = (torch.from_numpy(a).to(d) for a in (sc.x, sc.y, sc.z))
    L = _lib.load()
    p = narvis.points_struct((X, Y, Z))
    a = narvis.attrs_struct([])
    c = narvis.camera_struct(sc.cameras[0])
    keys = torch.empty(64 * 64, dtype=torch.int64, device=d)
    g = narvis.GBuffer(keys=keys)
    # larger than the static scratch: WORKSPACE before anything is enqueued
    st = L.narvis_rasterize_static(ctypes.byref(p), ctypes.byref(a), 4096, ctypes.byref(c), 3841, 2160,
                                   ctypes.byref(g.struct()), None)
    assert st == -5
    # a caller scratch is not taken by this call
    g2 = narvis.GBuffer(keys=keys, bounds=narvis.raster_bounds(64, 64, d))
    st = L.narvis_rasterize_static(ctypes.byref(p), ctypes.byref(a), 4096, ctypes.byref(c), 64, 64,
                                   ctypes.byref(g2.struct()), None)
    assert st == -1
