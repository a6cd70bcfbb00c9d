"""Full-size parity: the vector-field (50 M points) and trajectory (350 M
points) workloads at 1920x1080, rendered with the automatic launch
configuration the benchmark times, compared element by element with the CPU
oracle run on the same inputs."""
import time

import numpy as np
import pytest

from oracle import camera as ocam
from oracle import raster as orast
from paper_2407_19097_amd import narvis, scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def run_pair(sc, cams, with_planes=True, hinted=False):
    """hinted: each frame after the first gets the previous frame's keys as
    the hint of its bounded render (a viewer loop)."""
    n, W, H = sc.n, sc.W, sc.H
    t0 = time.time()
    xh, yh, zh = (t.cpu().numpy() for t in (sc.x, sc.y, sc.z))
    ah = [a.cpu().numpy() for a in sc.attrs]
    if ah and ah[0].dtype == np.int16:
        ah[0] = ah[0].view(np.uint16)
    print(f"  host copy {time.time() - t0:.1f}s", flush=True)
    inv = np.float32(1.0 / (sc.lut_max - sc.lut_min))
    lut = scenes.colour_lut()
    with_planes = with_planes and sc.lut_attr >= 0
    prev = None
    for cam in cams:
        g = narvis.GBuffer.allocate(W, H, nattr=len(sc.attrs), rgb=with_planes, vel2d=with_planes and sc.vel_attr >= 0)
        g.hint = prev if hinted else None
        if with_planes:
            g.lut = torch.from_numpy(lut).cuda()
            g.lut_attr, g.lut_min, g.lut_inv_range, g.vel_attr = sc.lut_attr, sc.lut_min, float(inv), sc.vel_attr
        narvis.narvis_rasterize((sc.x, sc.y, sc.z), sc.attrs, n, cam, W, H, g)
        torch.cuda.synchronize()
        keys = g.keys.cpu().numpy().view(np.uint64)
        t0 = time.time()
        M, near, far = ocam.clip_matrix(cam, W, H)
        okeys = orast.render(xh, yh, zh, M, near, far, W, H)
        print(f"  oracle render {time.time() - t0:.1f}s, covered {(okeys != orast.EMPTY).mean():.3f}", flush=True)
        np.testing.assert_array_equal(keys, okeys)
        o = orast.resolve(okeys, W, H, xh, yh, zh, M, ah, lut=lut if with_planes else None,
                          lut_attr=sc.lut_attr, lut_min=sc.lut_min, lut_inv_range=inv,
                          vel_attr=sc.vel_attr if with_planes else -1)
        np.testing.assert_array_equal(g.depth.cpu().numpy().view(np.uint32), o["depth"].view(np.uint32))
        np.testing.assert_array_equal(g.attr.cpu().numpy().view(np.uint32), o["attrs"].view(np.uint32))
        if with_planes:
            np.testing.assert_array_equal(g.rgb.cpu().numpy().view(np.uint32), o["rgb"].view(np.uint32))
        if "vel2d" in o:
            v = g.vel2d.cpu().numpy()
            for c in (0, 1, 3):
                np.testing.assert_array_equal(v[c].view(np.uint32), o["vel2d"][c].view(np.uint32))
            d = np.abs(v[2].view(np.int32).astype(np.int64) - o["vel2d"][2].view(np.int32).astype(np.int64))
            assert d.max() <= 4
        prev = g.keys
        del g


def test_vector_field_50m_full():
    announce("vector field 500x500x200 = 50M points, 1920x1080, orbit frames 0, 17, 45")
    sc = scenes.vector_field(device="cuda")
    run_pair(sc, [sc.cameras[0], sc.cameras[17], sc.cameras[45]])
    announce("vector field, orbit frames 17, 18, 19 with the previous frame's keys as hint")
    run_pair(sc, [sc.cameras[17], sc.cameras[18], sc.cameras[19]], hinted=True)


def test_trajectories_350m_full():
    announce("trajectories 3.5M particles x 100 steps = 350M points, 1920x1080, fly-through frame 60 + overview")
    sc = scenes.trajectories(device="cuda")
    run_pair(sc, [sc.cameras[60], sc.cameras[-1]], with_planes=True)
    announce("trajectories, fly-through frames 30, 31 with the previous frame's keys as hint")
    run_pair(sc, [sc.cameras[30], sc.cameras[31]], with_planes=False, hinted=True)


def test_terrain_1b_full_and_quarter():
    announce("terrain 1B points (RGBA u8, strided AoS views), 3840x2160, and its every-4th-point variant")
    from paper_2407_19097_amd import scenes as sc_mod
    sc = sc_mod.terrain(device="cuda")
    run_pair(sc, [sc.cameras[0]], with_planes=False)
    quarter = sc_mod.subsample(sc, 4)
    del sc
    run_pair(quarter, [quarter.cameras[0]], with_planes=False)
