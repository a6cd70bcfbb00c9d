"""Morton layout and batch-culled render against the CPU oracles.

The layout itself (order, original indices, per-batch boxes) is compared
element by element with oracle/layout.py; the render over a layout must give
the key buffer of the CPU raster oracle over the points in their ORIGINAL
order, bit for bit (every key carries the original index, so ties still go
to the lowest original index), single pass and bounded, on ragged sizes,
non-finite points, cameras inside and outside the cloud, equal-depth ties
whose Morton order is the reverse of their index order, and the full-size
vector-field and trajectory workloads.  Each test prints its case first."""
import numpy as np
import pytest

from oracle import camera as ocam
from oracle import layout as olay
from oracle import raster as orast
from paper_2407_19097_amd import narvis, scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_layout(x, y, z, sample=True):
    n = int(x.shape[0])
    X, Y, Z = dev(x), dev(y), dev(z)
    L = narvis.build_layout((X, Y, Z), n, sample=sample)
    torch.cuda.synchronize()
    return (X, Y, Z), L


def check_layout(x, y, z, L):
    n = int(x.shape[0])
    perm, boxes = olay.layout(x, y, z, batch=narvis.LAYOUT_BATCH)
    gi = L.index[:n].cpu().numpy().view(np.uint32)
    assert np.array_equal(gi, perm)
    for a, t in zip((x, y, z), (L.x, L.y, L.z)):
        assert np.array_equal(t[:n].cpu().numpy().view(np.uint32), a[perm].view(np.uint32))
    gb = L.boxes[:boxes.shape[0]].cpu().numpy()
    assert np.array_equal(gb[:, 0:3], boxes[:, 0]) and np.array_equal(gb[:, 4:7], boxes[:, 1])
    if L.sample:
        sidx, sboxes = olay.depth_sample(x, y, z, perm, batch=narvis.LAYOUT_BATCH)
        ns = sidx.shape[0]
        assert np.array_equal(L.sindex[:ns].cpu().numpy().view(np.uint32), sidx)
        for a, t in zip((x, y, z), (L.sx, L.sy, L.sz)):
            assert np.array_equal(t[:ns].cpu().numpy().view(np.uint32), a[sidx].view(np.uint32))
        gs = L.sboxes[:sboxes.shape[0]].cpu().numpy()
        assert np.array_equal(gs[:, 0:3], sboxes[:, 0]) and np.array_equal(gs[:, 4:7], sboxes[:, 1])


def render_layout(L, n, cam, W, H, bounded):
    vp, nf, ff = narvis.narvis_camera_matrix(cam, W, H)
    keys = torch.empty(W * H, dtype=torch.int64, device="cuda")
    narvis.narvis_raster_clear(keys, W, H)
    b = narvis.raster_bounds(W, H) if bounded else None
    narvis.narvis_raster_render_layout(L, n, vp, nf, ff, W, H, keys, bounds=b)
    torch.cuda.synchronize()
    return keys.cpu().numpy().view(np.uint64)


def oracle_keys(x, y, z, cam, W, H):
    M, near, far = ocam.clip_matrix(cam, W, H)
    return orast.render(x, y, z, M, near, far, W, H)


CAMS = [scenes.Camera(eye=(2, 2, 2), target=(0.5, 0.5, 0.5)),
        scenes.Camera(eye=(0.5, 0.5, 0.5), target=(1.0, 0.8, 0.2)),   # inside the cloud
        scenes.Camera(eye=(-3, 0.5, 0.5), target=(-6, 0.5, 0.5)),      # looking away: nothing kept
        scenes.Camera(eye=(0.5, -0.2, 0.55), target=(0.5, 1.0, 0.45), fovy_deg=30.0)]


@pytest.mark.parametrize("n", [1, 3, 4097, 65537, 300001])
def test_layout_build_matches_oracle(n):
    announce(f"layout build, unit cube n={n} with non-finite points")
    rng = np.random.default_rng(n)
    x, y, z = rng.random((3, n), dtype=np.float32)
    if n > 100:
        x[rng.integers(0, n, 20)] = np.nan
        z[rng.integers(0, n, 20)] = -np.inf
    _, L = gpu_layout(x, y, z)
    check_layout(x, y, z, L)


def test_layout_build_degenerate_extent():
    announce("layout build: every point on one plane and one line (zero extents)")
    n = 10000
    rng = np.random.default_rng(1)
    x = np.full(n, 0.25, np.float32)
    y = rng.random(n, dtype=np.float32)
    z = np.full(n, -2.0, np.float32)
    _, L = gpu_layout(x, y, z)
    check_layout(x, y, z, L)


@pytest.mark.parametrize("bounded,sample", [(False, True), (True, True), (True, False)])
@pytest.mark.parametrize("n", [4097, 300001, 1_000_003])
def test_layout_render_matches_oracle(n, bounded, sample):
    announce(f"layout render vs oracle (original order), unit cube n={n}, bounded={bounded}, depth sample={sample}, "
             "4 cameras")
    rng = np.random.default_rng(7 + n)
    x, y, z = rng.random((3, n), dtype=np.float32)
    x[rng.integers(0, n, 30)] = np.nan
    _, L = gpu_layout(x, y, z, sample=sample)
    for cam in CAMS:
        for W, H in ((320, 240), (97, 131)):
            got = render_layout(L, n, cam, W, H, bounded)
            want = oracle_keys(x, y, z, cam, W, H)
            assert np.array_equal(got, want), (cam, W, H)


@pytest.mark.parametrize("bounded", [False, True])
def test_layout_equal_depth_ties_in_reverse_morton_order(bounded):
    """Identity view (eye at the origin looking down -z, 90 degree field of
    view, so M00 = M11 = 1 and w = -z exactly): groups of points at one depth
    share a pixel but lie in different Morton cells, and their original
    indices run against the Morton order, so the lowest index is the last in
    layout order; the winner must still be the lowest original index."""
    announce(f"layout render: equal-depth ties against the Morton order, bounded={bounded}")
    W = H = 64
    cam = scenes.Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fovy_deg=90.0)
    rng = np.random.default_rng(5)
    xs, ys, zs = [], [], []
    # 3000 groups of 8 points; inside a group same pixel, same depth, x cells increasing
    for g in range(3000):
        px, py = rng.integers(0, W), rng.integers(0, H)
        d = np.float32(rng.choice([1.0, 1.5, 2.0]))
        x0 = ((px + 0.05) / W * 2.0 - 1.0) * d
        y0 = (1.0 - (py + 0.5) / H * 2.0) * d
        for k in range(8):
            xs.append(np.float32(x0 + k * 0.1 / W * 2.0 * d))
            ys.append(np.float32(y0))
            zs.append(-d)
    # index order = reverse of the x order inside each group
    x = np.array(xs, np.float32).reshape(-1, 8)[:, ::-1].reshape(-1).copy()
    y = np.array(ys, np.float32).reshape(-1, 8)[:, ::-1].reshape(-1).copy()
    z = np.array(zs, np.float32).reshape(-1, 8)[:, ::-1].reshape(-1).copy()
    # two corner points fix the cloud's box: x cells of 4/1024, finer than
    # the points' spacing in a group at these depths
    x = np.concatenate([x, np.float32([-2, 2])])
    y = np.concatenate([y, np.float32([-2, 2])])
    z = np.concatenate([z, np.float32([-2, -0.5])])
    n = x.shape[0]
    _, L = gpu_layout(x, y, z)
    perm = L.index[:n].cpu().numpy().view(np.uint32)
    assert not np.array_equal(perm, np.sort(perm))  # the layout does reorder
    got = render_layout(L, n, cam, W, H, bounded)
    want = oracle_keys(x, y, z, cam, W, H)
    assert np.array_equal(got, want)
    assert (want != orast.EMPTY).sum() > 1000


def test_layout_whole_frame_planes():
    announce("narvis_rasterize_layout vs narvis_rasterize: keys and every plane, unit cube 1M at 640x480")
    sc = scenes.unit_cube(n=1_000_000, seed=4, W=640, H=480)
    P = tuple(dev(a) for a in (sc.x, sc.y, sc.z))
    A = [dev(a) for a in sc.attrs]
    L = narvis.build_layout(P, sc.n)
    lut = dev(scenes.colour_lut())
    out = []
    for use_layout in (False, True):
        g = narvis.GBuffer.allocate(640, 480, nattr=4, rgb=True, vel2d=True)
        g.lut, g.lut_attr, g.lut_min, g.lut_inv_range, g.vel_attr = lut, 3, 0.0, float(np.float32(1 / 3.5)), 0
        if use_layout:
            narvis.narvis_rasterize_layout(L, P, A, sc.n, sc.cameras[0], 640, 480, g)
        else:
            narvis.narvis_rasterize(P, A, sc.n, sc.cameras[0], 640, 480, g)
        torch.cuda.synchronize()
        out.append({k: getattr(g, k).cpu().numpy().view(np.uint32) for k in ("keys", "depth", "attr", "rgb", "vel2d")})
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def full_size(sc, cams):
    n, W, H = sc.n, sc.W, sc.H
    xh, yh, zh = (t.cpu().numpy() for t in (sc.x, sc.y, sc.z))
    L = narvis.build_layout((sc.x, sc.y, sc.z), n)
    torch.cuda.synchronize()
    print(f"  layout built for {n} points", flush=True)
    for cam in cams:
        got = render_layout(L, n, cam, W, H, bounded=True)
        want = oracle_keys(xh, yh, zh, cam, W, H)
        print(f"  covered {(want != orast.EMPTY).mean():.3f}", flush=True)
        assert np.array_equal(got, want)
    del L
    torch.cuda.empty_cache()


def test_layout_vector_field_50m_full():
    announce("layout render, vector field 50M points at 1920x1080, orbit frames 0 and 31")
    sc = scenes.vector_field(device="cuda")
    full_size(sc, [sc.cameras[0], sc.cameras[31]])


def test_layout_trajectories_350m_full():
    announce("layout render, trajectories 350M points at 1920x1080, overview and fly-through frames 0, 60")
    sc = scenes.trajectories(device="cuda")
    full_size(sc, [sc.cameras[-1], sc.cameras[0], sc.cameras[60]])
