"""GPU render/resolve vs the CPU oracle, element by element (bit-exact on keys,
depth and every G-buffer plane except theta, which is within 4 ulp).

Each test prints the case it runs before touching the GPU."""
import math

import numpy as np
import pytest

from oracle import camera as ocam
from oracle import raster as orast
from paper_2407_19097_amd import narvis, scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def ulp_diff(a, b):
    """ulps between two float32 arrays (sign-magnitude aware)."""
    ia = a.view(np.int32).astype(np.int64)
    ib = b.view(np.int32).astype(np.int64)
    ia = np.where(ia < 0, -(ia & 0x7FFFFFFF), ia)
    ib = np.where(ib < 0, -(ib & 0x7FFFFFFF), ib)
    return np.abs(ia - ib)


def gpu_frame(x, y, z, attrs, cam, W, H, lut=None, lut_attr=-1, lut_min=0.0, lut_inv=1.0, vel_attr=-1,
              variant=0, grid_blocks=0, xyz_dev=None, attrs_dev=None, bounded=False):
    """Clear + render + resolve through the C ABI; returns numpy planes
    (and the tile bounds of the bounded render when it is asked for)."""
    n = int(x.shape[0])
    vp, nf, ff = narvis.narvis_camera_matrix(cam, W, H)
    X, Y, Z = xyz_dev if xyz_dev is not None else (dev(x), dev(y), dev(z))
    A = attrs_dev if attrs_dev is not None else [dev(a) for a in attrs]
    g = narvis.GBuffer.allocate(W, H, nattr=len(A), depth=True, rgb=lut is not None, vel2d=vel_attr >= 0)
    if lut is not None:
        g.lut = dev(lut)
        g.lut_attr, g.lut_min, g.lut_inv_range = lut_attr, lut_min, lut_inv
    g.vel_attr = vel_attr
    narvis.narvis_raster_clear(g.keys, W, H)
    narvis.narvis_raster_render((X, Y, Z), n, vp, nf, ff, W, H, g.keys, variant=variant, grid_blocks=grid_blocks,
                                bounds=g.bounds if bounded else None)
    narvis.narvis_raster_resolve((X, Y, Z), A, n, vp, W, H, g)
    out = {"keys": host(g.keys).view(np.uint64), "depth": host(g.depth)}
    if bounded:
        out["bounds"] = host(g.bounds).view(np.uint16)
    if g.attr is not None:
        out["attrs"] = host(g.attr)
    if g.rgb is not None:
        out["rgb"] = host(g.rgb)
    if g.vel2d is not None:
        out["vel2d"] = host(g.vel2d)
    return out


def oracle_frame(x, y, z, attrs, cam, W, H, lut=None, lut_attr=-1, lut_min=0.0, lut_inv=1.0, vel_attr=-1):
    M, near, far = ocam.clip_matrix(cam, W, H)
    keys = orast.render(x, y, z, M, near, far, W, H)
    out = orast.resolve(keys, W, H, x, y, z, M, attrs, lut=lut, lut_attr=lut_attr, lut_min=lut_min,
                        lut_inv_range=lut_inv, vel_attr=vel_attr)
    out["keys"] = keys
    return out


def assert_same(g, o, theta_ulps=4):
    np.testing.assert_array_equal(g["keys"], o["keys"])
    np.testing.assert_array_equal(g["depth"].view(np.uint32), o["depth"].view(np.uint32))
    if "attrs" in o:
        np.testing.assert_array_equal(g["attrs"].view(np.uint32), o["attrs"].view(np.uint32))
    if "rgb" in o:
        np.testing.assert_array_equal(g["rgb"].view(np.uint32), o["rgb"].view(np.uint32))
    if "vel2d" in o:
        for c in (0, 1, 3):
            np.testing.assert_array_equal(g["vel2d"][c].view(np.uint32), o["vel2d"][c].view(np.uint32))
        d = ulp_diff(g["vel2d"][2], o["vel2d"][2])
        assert int(d.max(initial=0)) <= theta_ulps, f"theta differs by {int(d.max())} ulp"


def scene_args(sc):
    inv = 1.0 / (sc.lut_max - sc.lut_min) if sc.lut_attr >= 0 else 1.0
    return dict(lut=scenes.colour_lut() if sc.lut_attr >= 0 else None, lut_attr=sc.lut_attr,
                lut_min=sc.lut_min, lut_inv=np.float32(inv), vel_attr=sc.vel_attr)


def test_unit_cube_full_parity():
    announce("unit cube 1M points 512x512, all planes")
    sc = scenes.unit_cube()
    kw = scene_args(sc)
    g = gpu_frame(sc.x, sc.y, sc.z, sc.attrs, sc.cameras[0], sc.W, sc.H, **kw)
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, sc.cameras[0], sc.W, sc.H, **kw)
    assert (o["keys"] != EMPTY).sum() > 0.15 * sc.W * sc.H
    assert_same(g, o)


@pytest.mark.parametrize("bounded", [False, True])
@pytest.mark.parametrize("znear", [1e-39, 0.1])
def test_both_division_paths(znear, bounded):
    """The render divides by the depth through a correctly rounded reciprocal
    when the fp32 cull range lies in [2^-124, 2^125) (znear 0.1), by IEEE
    division otherwise (a denormal znear): both bit-exact, single-pass and
    bounded."""
    announce(f"unit cube 200003 points 301x207, LDS render, znear={znear}, bounded={bounded}")
    sc = scenes.unit_cube(n=200003, seed=5, W=301, H=207)
    cam = scenes.Camera(eye=(1.7, 1.5, 1.3), target=(0.5, 0.5, 0.5), znear=znear)
    kw = scene_args(sc)
    g = gpu_frame(sc.x, sc.y, sc.z, sc.attrs, cam, sc.W, sc.H, variant=3, bounded=bounded, **kw)
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, cam, sc.W, sc.H, **kw)
    assert (o["keys"] != EMPTY).mean() > 0.1
    assert_same(g, o)


@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1023, 4097, 65537, 300001])
def test_ragged_sizes(n):
    announce(f"ragged n={n} 97x61")
    sc = scenes.unit_cube(n=max(n, 1), seed=n + 1, W=97, H=61)
    x, y, z = sc.x[:n], sc.y[:n], sc.z[:n]
    attrs = [a[:n] for a in sc.attrs]
    kw = scene_args(sc)
    cam = scenes.Camera(eye=(1.6, 1.4, 1.2), target=(0.5, 0.5, 0.5), up=(0.2, 0.1, 1.0))
    g = gpu_frame(x, y, z, attrs, cam, sc.W, sc.H, **kw)
    o = oracle_frame(x, y, z, attrs, cam, sc.W, sc.H, **kw)
    assert_same(g, o)


@pytest.mark.parametrize("variant", [1, 2, 3])
@pytest.mark.parametrize("grid", [0, 1, 7, 8, 100])
def test_variants_and_launch_geometry(variant, grid):
    announce(f"variant={variant} grid_blocks={grid}")
    sc = scenes.unit_cube(n=200003, seed=9, W=160, H=90)
    cam = scenes.Camera(eye=(1.8, 1.5, 1.3), target=(0.5, 0.5, 0.5))
    g = gpu_frame(sc.x, sc.y, sc.z, sc.attrs, cam, sc.W, sc.H, variant=variant, grid_blocks=grid)
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, cam, sc.W, sc.H)
    assert_same(g, o)


def expected_bounds(x, y, z, cam, W, H):
    """Bounds the bounded render must leave behind, from the oracle: the keys
    of its first level (points of every 8th chunk of 2048, plus the last n % 4
    points; the others are made NaN so that the indices stay put), then per
    tile of 2^s x 2^s pixels (smallest s >= 3 with at most 8192 tiles) the
    largest depth bits over the tile's pixels shifted down by 16, and per
    pixel its depth bits.  Returns (tile bounds, pixel bounds)."""
    n = len(x)
    i = np.arange(n)
    sample = ((i // 2048) % 8 == 0) | (i >= 4 * (n // 4))
    xs = np.where(sample, x, np.float32(np.nan)).astype(np.float32)
    M, near, far = ocam.clip_matrix(cam, W, H)
    keys = orast.render(xs, y, z, M, near, far, W, H)
    s = 3
    while -(-W >> s) * -(-H >> s) > 8192:
        s += 1
    tx, ty = -(-W >> s), -(-H >> s)
    depth = np.full((ty << s, tx << s), 0, np.uint64)
    depth[:H, :W] = (keys >> np.uint64(32)).reshape(H, W)
    tiles = depth.reshape(ty, 1 << s, tx, 1 << s).max(axis=(1, 3)).reshape(-1)
    return (tiles >> np.uint64(16)).astype(np.uint16), (keys >> np.uint64(32)).astype(np.uint32)


@pytest.mark.parametrize("n,W,H,grid", [(4096, 64, 48, 0), (4099, 97, 61, 0), (65537, 32, 24, 1),
                                        (300001, 97, 61, 7), (300001, 301, 207, 0),
                                        (1 << 20, 160, 120, 0), (1 << 20, 1920, 1080, 100)])
def test_bounded_render(n, W, H, grid):
    """Bounded two-pass render (sample chunks, tile bounds, the rest culled
    against them): keys and planes bit-exact, and the bounds exactly those
    of the oracle's sample pass."""
    announce(f"bounded render n={n} {W}x{H} grid_blocks={grid}")
    sc = scenes.unit_cube(n=n, seed=n % 97 + W, W=W, H=H)
    cam = scenes.Camera(eye=(1.7, 1.5, 1.3), target=(0.5, 0.5, 0.5))
    kw = scene_args(sc)
    g = gpu_frame(sc.x, sc.y, sc.z, sc.attrs, cam, W, H, variant=3, grid_blocks=grid, bounded=True, **kw)
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, cam, W, H, **kw)
    assert_same(g, o)
    exp, exp_pix = expected_bounds(sc.x, sc.y, sc.z, cam, W, H)
    np.testing.assert_array_equal(g["bounds"][:len(exp)], exp)
    np.testing.assert_array_equal(g["bounds"][8192:].view(np.uint32)[:W * H], exp_pix)
    if n >= 20 * W * H:
        assert (exp < 0xFFFF).mean() > 0.1  # dense enough that the culling is exercised


def test_hinted_bounded_render():
    """The hinted render equals the oracle whatever the hint holds: the keys
    of another camera's frame (the viewer-loop use), the frame's own keys,
    random keys with indices past n, and an empty buffer; the hint is read
    only."""
    announce("hinted bounded render, 1M points + ragged tail, 200x150")
    n, W, H = (1 << 20) + 1234 + 3, 200, 150
    sc = scenes.unit_cube(n=n, seed=41, W=W, H=H)
    cams = [scenes.Camera(eye=(1.9, 1.4, 1.2), target=(0.5, 0.5, 0.5)),
            scenes.Camera(eye=(1.7, 1.7, 1.1), target=(0.5, 0.5, 0.45))]
    X, Y, Z = dev(sc.x), dev(sc.y), dev(sc.z)
    bounds = narvis.raster_bounds(W, H)
    keys = torch.empty(W * H, dtype=torch.int64, device="cuda")
    okeys = []
    for cam in cams:
        M, near, far = ocam.clip_matrix(cam, W, H)
        okeys.append(orast.render(sc.x, sc.y, sc.z, M, near, far, W, H))
    rng = np.random.default_rng(5)
    junk = rng.integers(0, (1 << 63) - 1, size=W * H, dtype=np.int64)
    junk[::3] = -1                                              # empty keys
    junk[1::3] = (junk[1::3] & ~0xFFFFFFFF) | (n + 7)           # indices past n
    hints = {"other camera": torch.from_numpy(okeys[0].view(np.int64)).cuda(),
             "own frame": torch.from_numpy(okeys[1].view(np.int64)).cuda(),
             "random": torch.from_numpy(junk).cuda(),
             "empty": torch.full((W * H,), -1, dtype=torch.int64, device="cuda")}
    vp, nf, ff = narvis.narvis_camera_matrix(cams[1], W, H)
    for name, hint in hints.items():
        before = hint.clone()
        narvis.narvis_raster_clear(keys, W, H)
        narvis.narvis_raster_render((X, Y, Z), n, vp, nf, ff, W, H, keys, variant=3, bounds=bounds, hint_keys=hint)
        np.testing.assert_array_equal(host(keys).view(np.uint64), okeys[1], err_msg=name)
        assert torch.equal(hint, before), name


def test_bounded_render_merges_into_existing_keys():
    """Keys are merged into what the buffer holds: the bounded render of all
    the points onto a buffer that already holds the first half's keys (its
    bounds then start from those keys) gives the keys of all the points."""
    announce("bounded render onto the first half's keys, 1M points 160x120")
    n, W, H = 1 << 20, 160, 120
    sc = scenes.unit_cube(n=n, seed=31, W=W, H=H)
    cam = scenes.Camera(eye=(1.7, 1.5, 1.3), target=(0.5, 0.5, 0.5))
    vp, nf, ff = narvis.narvis_camera_matrix(cam, W, H)
    X, Y, Z = dev(sc.x), dev(sc.y), dev(sc.z)
    keys = torch.empty(W * H, dtype=torch.int64, device="cuda")
    bounds = narvis.raster_bounds(W, H)
    h = n // 2
    narvis.narvis_raster_clear(keys, W, H)
    narvis.narvis_raster_render((X[:h], Y[:h], Z[:h]), h, vp, nf, ff, W, H, keys, variant=3, bounds=bounds)
    part = host(keys).view(np.uint64).copy()
    narvis.narvis_raster_clear(keys, W, H)
    narvis.narvis_raster_render((X, Y, Z), n, vp, nf, ff, W, H, keys, variant=3, bounds=bounds)
    full = host(keys).view(np.uint64).copy()
    # onto the first half's keys
    keys.copy_(torch.from_numpy(part.view(np.int64)).cuda())
    narvis.narvis_raster_render((X, Y, Z), n, vp, nf, ff, W, H, keys, variant=3, bounds=bounds)
    merged = host(keys).view(np.uint64)
    M, near, far = ocam.clip_matrix(cam, W, H)
    okeys = orast.render(sc.x, sc.y, sc.z, M, near, far, W, H)
    np.testing.assert_array_equal(full, okeys)
    np.testing.assert_array_equal(merged, okeys)
    ohalf = orast.render(sc.x[:h], sc.y[:h], sc.z[:h], M, near, far, W, H)
    np.testing.assert_array_equal(part, ohalf)


def test_bounded_render_descending_depth_one_pixel():
    """Every later point closer than all earlier ones, all in one pixel: the
    bounds cull nothing that could win."""
    announce("bounded render, 1M points in one pixel, descending depth")
    n = 1 << 20
    cam = scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0))
    z = -np.linspace(5.0, 1.0, n, dtype=np.float32)
    x = np.full(n, 0.001, np.float32)
    y = np.full(n, 0.001, np.float32)
    g = gpu_frame(x, y, z, [], cam, 16, 16, variant=3, bounded=True)
    o = oracle_frame(x, y, z, [], cam, 16, 16)
    assert_same(g, o)


def test_unaligned_points_take_scalar_path():
    announce("unaligned point arrays (offset by one element)")
    sc = scenes.unit_cube(n=100001, seed=4, W=64, H=64)
    cam = sc.cameras[0]
    X, Y, Z = dev(sc.x), dev(sc.y), dev(sc.z)
    x1, y1, z1 = X[1:], Y[1:], Z[1:]
    g = gpu_frame(sc.x[1:], sc.y[1:], sc.z[1:], [], cam, 64, 64, xyz_dev=(x1, y1, z1), attrs_dev=[])
    o = oracle_frame(sc.x[1:], sc.y[1:], sc.z[1:], [], cam, 64, 64)
    assert_same(g, o)


def test_adversarial_points():
    announce("adversarial: ties, borders, non-finite, behind camera, near/far")
    W, H = 40, 30
    cam = scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0), fovy_deg=70.0)
    M, near, far = ocam.clip_matrix(cam, W, H)
    m0, m1 = float(M[0]), float(M[5])
    pts = [(0, 0, -1), (0, 0, -1), (0.01, 0.01, -2), (0.01, 0.01, -2),  # exact ties
           (1.0, 0, -m0), (-1.0, 0, -m0), (0, 1.0, -m1), (0, -1.0, -m1),  # borders
           (np.nan, 0, -1), (0, np.inf, -1), (0, 0, np.nan), (0, 0, -np.inf), (0, 0, 1), (0, 0, 0),
           (0, 0, -float(near)), (0, 0, -float(np.nextafter(near, np.float32(0)))),
           (0, 0, -float(far)), (0.3, 0.2, -float(np.nextafter(far, np.float32(np.inf))))]
    rng = np.random.default_rng(1)
    extra = (rng.random((5000, 3)) * np.array([2, 2, -3]) - np.array([1, 1, 0.1])).tolist()
    pts = np.array(pts + extra + [(0, 0, -1)] * 100, np.float32)
    x, y, z = (np.ascontiguousarray(pts[:, k]) for k in range(3))
    a = [np.arange(len(x), dtype=np.float32)]
    g = gpu_frame(x, y, z, a, cam, W, H)
    o = oracle_frame(x, y, z, a, cam, W, H)
    assert_same(g, o)


def test_all_points_in_one_pixel():
    announce("all points in one pixel, 1M points, descending depth")
    n = 1 << 20
    W, H = 16, 16
    cam = scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0))
    z = -np.linspace(5.0, 1.0, n, dtype=np.float32)  # later points closer: worst case for early-z
    x = np.full(n, 0.001, np.float32)
    y = np.full(n, 0.001, np.float32)
    g = gpu_frame(x, y, z, [], cam, W, H)
    o = oracle_frame(x, y, z, [], cam, W, H)
    assert_same(g, o)


def test_attribute_formats_and_strides():
    announce("u8/u16/f16/f32 attributes, AoS strides, NaN halves")
    sc = scenes.unit_cube(n=120000, seed=6, W=128, H=96)
    n = sc.n
    rng = np.random.default_rng(2)
    rgba = rng.integers(0, 256, size=(n, 4), dtype=np.uint8)
    u16 = rng.integers(0, 65536, size=n, dtype=np.uint16)
    halfs = rng.standard_normal(n).astype(np.float16)
    halfs[::97] = np.float16(np.nan)
    halfs[1::97] = np.array([0x7C01], np.uint16).view(np.float16)[0]  # signalling NaN
    halfs[2::97] = np.float16(6e-8)  # subnormal
    halfs[3::97] = -np.float16(np.inf)
    pair = rng.standard_normal((n, 2)).astype(np.float32)
    RGBA = dev(rgba)
    PAIR = dev(pair)
    attrs_dev = [RGBA[:, 0], RGBA[:, 3], dev(u16), dev(halfs), PAIR[:, 1], dev(sc.attrs[3])]
    attrs_host = [rgba[:, 0], rgba[:, 3], u16, halfs, pair[:, 1], sc.attrs[3]]
    cam = scenes.Camera(eye=(1.7, 1.2, 1.5), target=(0.5, 0.5, 0.5))
    kw = dict(lut=scenes.colour_lut(), lut_attr=3, lut_min=-2.0, lut_inv=np.float32(0.25))
    g = gpu_frame(sc.x, sc.y, sc.z, attrs_host, cam, sc.W, sc.H, attrs_dev=attrs_dev, **kw)
    o = oracle_frame(sc.x, sc.y, sc.z, attrs_host, cam, sc.W, sc.H, **kw)
    assert_same(g, o)


def test_eight_attributes_and_velocity_planes():
    announce("eight attributes, Vel2D from a tilted camera")
    sc = scenes.unit_cube(n=250000, seed=8, W=200, H=150)
    attrs = list(sc.attrs) + [a * np.float32(k + 2) for k, a in enumerate(sc.attrs)]
    cam = scenes.Camera(eye=(2.0, 1.8, 1.6), target=(0.5, 0.5, 0.5), up=(0.3, -0.4, 1.0))
    kw = dict(lut=scenes.colour_lut(), lut_attr=7, lut_min=0.0, lut_inv=np.float32(0.1), vel_attr=4)
    g = gpu_frame(sc.x, sc.y, sc.z, attrs, cam, sc.W, sc.H, **kw)
    o = oracle_frame(sc.x, sc.y, sc.z, attrs, cam, sc.W, sc.H, **kw)
    assert_same(g, o)


def test_rasterize_whole_frame_entry_point():
    announce("narvis_rasterize (camera -> clear -> render -> resolve)")
    sc = scenes.unit_cube(n=300000, seed=12, W=256, H=192)
    kw = scene_args(sc)
    X, Y, Z = dev(sc.x), dev(sc.y), dev(sc.z)
    A = [dev(a) for a in sc.attrs]
    g = narvis.GBuffer.allocate(sc.W, sc.H, nattr=4, rgb=True, vel2d=True)
    g.lut = dev(kw["lut"])
    g.lut_attr, g.lut_min, g.lut_inv_range, g.vel_attr = 3, 0.0, float(kw["lut_inv"]), 0
    g.keys.fill_(12345)  # stale contents must be cleared by the call
    narvis.narvis_rasterize((X, Y, Z), A, sc.n, sc.cameras[0], sc.W, sc.H, g)
    got = {"keys": host(g.keys).view(np.uint64), "depth": host(g.depth), "attrs": host(g.attr),
           "rgb": host(g.rgb), "vel2d": host(g.vel2d)}
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, sc.cameras[0], sc.W, sc.H, **kw)
    assert_same(got, o)


def test_rasterize_with_previous_frame_hint():
    announce("narvis_rasterize of a second camera with the first frame's keys as hint")
    sc = scenes.unit_cube(n=300000, seed=13, W=256, H=192)
    kw = scene_args(sc)
    X, Y, Z = dev(sc.x), dev(sc.y), dev(sc.z)
    A = [dev(a) for a in sc.attrs]
    cam2 = scenes.Camera(eye=(1.9, 2.2, 1.7), target=(0.45, 0.5, 0.5))
    frames = []
    for k, cam in enumerate((sc.cameras[0], cam2)):
        g = narvis.GBuffer.allocate(sc.W, sc.H, nattr=4, rgb=True, vel2d=True)
        g.lut = dev(kw["lut"])
        g.lut_attr, g.lut_min, g.lut_inv_range, g.vel_attr = 3, 0.0, float(kw["lut_inv"]), 0
        g.hint = frames[-1].keys if frames else None
        narvis.narvis_rasterize((X, Y, Z), A, sc.n, cam, sc.W, sc.H, g)
        frames.append(g)
    g = frames[1]
    got = {"keys": host(g.keys).view(np.uint64), "depth": host(g.depth), "attrs": host(g.attr),
           "rgb": host(g.rgb), "vel2d": host(g.vel2d)}
    o = oracle_frame(sc.x, sc.y, sc.z, sc.attrs, cam2, sc.W, sc.H, **kw)
    assert_same(got, o)


def test_rgb8_colour_into_network_input_slices():
    """Terrain colours (AoS RGBA uint8) resolved in the RGB8 colour mode
    straight into the network's input tensor: rgb and depth are slices of one
    [8][H][W] buffer, bit-exact against the oracle; the velocity slices a
    scene without velocity leaves alone stay as the caller set them."""
    announce("terrain 90000 points 160x96, RGB8 rgb + depth into an [8][H][W] input")
    sc = scenes.terrain(device="cpu", grid=256, lattice=300, n=90000, W=160, H=96)
    x, y, z = (t.numpy() for t in (sc.x, sc.y, sc.z))
    rgba = sc.extra["rgba"].numpy()
    W, H, cam = sc.W, sc.H, sc.cameras[0]
    RGBA = dev(rgba)
    A = [RGBA[:, c] for c in range(4)]
    feat = torch.zeros((8, W * H), dtype=torch.float32, device="cuda")
    g = narvis.GBuffer(keys=torch.empty(W * H, dtype=torch.int64, device="cuda"), depth=feat[3], rgb=feat[0:3],
                       lut_attr=0, rgb_mode=narvis.COLOR_RGB8, bounds=narvis.raster_bounds(W, H, "cuda"))
    narvis.narvis_rasterize((dev(x), dev(y), dev(z)), A, x.shape[0], cam, W, H, g)
    got = host(feat)
    M, near, far = ocam.clip_matrix(cam, W, H)
    okeys = orast.render(x, y, z, M, near, far, W, H)
    o = orast.resolve(okeys, W, H, x, y, z, M, [rgba[:, c].copy() for c in range(4)], rgb_mode=1, lut_attr=0)
    assert (okeys != EMPTY).mean() > 0.3
    np.testing.assert_array_equal(host(g.keys).view(np.uint64), okeys)
    np.testing.assert_array_equal(got[0:3].view(np.uint32), o["rgb"].view(np.uint32))
    np.testing.assert_array_equal(got[3].view(np.uint32), o["depth"].view(np.uint32))
    assert (got[4:8] == 0).all()
