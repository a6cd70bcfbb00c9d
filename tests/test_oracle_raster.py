"""Pins for the CPU raster oracle (render + resolve, Sec. 3.2) against facts
that do not come from the oracle itself: a hand-derived fixture, brute-force
per-pixel nearest-depth search, exact FP64 projection, closed-form cameras,
border and tie rules, and library conversions."""
import math
import os

import numpy as np
import pytest

from oracle import camera as ocam
from oracle import raster as orast
from paper_2407_19097_amd import scenes

EMPTY = np.uint64(0xFFFFFFFFFFFFFFFF)
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def identity_camera(fovy=90.0):
    return scenes.Camera(eye=(0.0, 0.0, 0.0), target=(0.0, 0.0, -1.0), up=(0.0, 1.0, 0.0), fovy_deg=fovy)


def f32bits(v):
    return int(np.float32(v).view(np.uint32))


def load_golden():
    pts, expect, hdr = [], [], None
    with open(os.path.join(GOLDEN, "raster_tiny.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            tok = line.split()
            if tok[0] == "=":
                expect.append((int(tok[1]), int(tok[2]), float(tok[3]), float(tok[4])))
            elif hdr is None:
                hdr = tuple(int(t) for t in tok)
            else:
                pts.append([float(t) for t in tok[1:]])
    return hdr, np.array(pts, dtype=np.float32), expect


def test_golden_fixture():
    (W, H, fovy), pts, expect = load_golden()
    cam = identity_camera(fovy)
    M, near, far = ocam.clip_matrix(cam, W, H)
    assert M[0] == 1.0 and M[5] == 1.0 and list(M[12:16]) == [0.0, 0.0, -1.0, 0.0]
    keys = orast.render(pts[:, 0], pts[:, 1], pts[:, 2], M, near, far, W, H)
    want = np.full(W * H, EMPTY, dtype=np.uint64)
    for pix, idx, depth, _ in expect:
        want[pix] = np.uint64((f32bits(depth) << 32) | idx)
    np.testing.assert_array_equal(keys, want)
    out = orast.resolve(keys, W, H, pts[:, 0], pts[:, 1], pts[:, 2], M, [pts[:, 3].copy()])
    d = np.zeros(W * H, np.float32)
    a = np.zeros(W * H, np.float32)
    for pix, _, depth, attr in expect:
        d[pix], a[pix] = depth, attr
    np.testing.assert_array_equal(out["depth"], d)
    np.testing.assert_array_equal(out["attrs"][0], a)


def project_np(x, y, z, M, near, far, W, H):
    """Per-point pixel and depth in numpy float32, one rounded op at a time."""
    M = M.astype(np.float32)
    with np.errstate(all="ignore"):
        cx = ((M[0] * x + M[1] * y) + M[2] * z) + M[3]
        cy = ((M[4] * x + M[5] * y) + M[6] * z) + M[7]
        w = ((M[12] * x + M[13] * y) + M[14] * z) + M[15]
        ok = (w >= near) & (w <= far)
        nx = cx / w
        ny = cy / w
        sx = (nx * np.float32(0.5) + np.float32(0.5)) * np.float32(W)
        sy = (np.float32(0.5) - ny * np.float32(0.5)) * np.float32(H)
        ok &= (sx >= 0) & (sx < W) & (sy >= 0) & (sy < H)
    pix = np.where(ok, np.floor(np.where(ok, sy, 0)).astype(np.int64) * W
                   + np.floor(np.where(ok, sx, 0)).astype(np.int64), -1)
    return pix, w


def brute_force(x, y, z, M, near, far, W, H):
    """For every pixel scan all points; the winner is the lexicographic minimum
    of (depth as a float, index) among the points landing in it."""
    pix, w = project_np(x, y, z, M, near, far, W, H)
    win = np.full(W * H, -1, dtype=np.int64)
    for p in range(W * H):
        cand = np.nonzero(pix == p)[0]
        if cand.size:
            order = np.lexsort((cand, w[cand].astype(np.float64)))
            win[p] = cand[order[0]]
    return win, w


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_tiny(seed):
    rng = np.random.default_rng(100 + seed)
    n, W, H = 4000, 48, 32
    xyz = rng.random((3, n), dtype=np.float32)
    # quantise positions so that many points share a pixel and some share a depth exactly
    xyz = (np.round(xyz * 256) / 256).astype(np.float32)
    xyz[:, 1::5] = xyz[:, 0::5][:, : xyz[:, 1::5].shape[1]]  # exact duplicates
    cam = scenes.Camera(eye=(1.3, 1.1, 0.9), target=(0.5, 0.5, 0.5))
    M, near, far = ocam.clip_matrix(cam, W, H)
    keys = orast.render(xyz[0], xyz[1], xyz[2], M, near, far, W, H)
    win, w = brute_force(xyz[0], xyz[1], xyz[2], M, near, far, W, H)
    assert (win >= 0).sum() > W * H // 3
    for p in range(W * H):
        if win[p] < 0:
            assert keys[p] == EMPTY
        else:
            i = int(win[p])
            assert int(keys[p]) & 0xFFFFFFFF == i
            assert np.uint32(int(keys[p]) >> 32).view(np.float32) == w[i]


TILTED = [scenes.Camera(eye=(3.0, -2.0, 1.5), target=(0.2, 0.4, 0.1)),
          scenes.Camera(eye=(-1.0, 2.5, 0.7), target=(0.5, 0.3, 0.6), up=(0.4, -0.3, 1.0)),
          scenes.Camera(eye=(0.4, 0.6, 3.0), target=(0.5, 0.5, 0.0), up=(1.0, 0.2, 0.1))]


@pytest.mark.parametrize("cam", TILTED)
def test_projection_matches_exact_fp64(cam):
    """Away from pixel borders the pixel equals the one given by exact real
    arithmetic on the fp32 matrix, and the depth is the view-axis distance."""
    rng = np.random.default_rng(7)
    W, H = 640, 360
    M, near, far = ocam.clip_matrix(cam, W, H)
    Md = M.astype(np.float64).reshape(4, 4)
    pts = (rng.random((3, 20000)) * 2 - 0.5).astype(np.float32)
    checked = 0
    eye = np.array(cam.eye)
    f = np.array(cam.target) - eye
    f /= np.linalg.norm(f)
    for k in range(pts.shape[1]):
        p = pts[:, k].astype(np.float64)
        c = Md @ np.append(p, 1.0)
        sx = (c[0] / c[3] * 0.5 + 0.5) * W
        sy = (0.5 - c[1] / c[3] * 0.5) * H
        pix, w = orast.project_point(M, near, far, W, H, *pts[:, k])
        inside = 0 <= sx < W and 0 <= sy < H and near <= c[3] <= far
        dist = min(abs(sx - round(sx)), abs(sy - round(sy)))
        if dist < 1e-3 or abs(sx) < 1e-3 or abs(sy) < 1e-3:
            continue
        if inside:
            assert pix == int(math.floor(sy)) * W + int(math.floor(sx))
            assert abs(float(w) - c[3]) <= 4e-7 * abs(c[3])
            # depth is the distance along the viewing direction
            assert abs(float(w) - float((p - eye) @ f)) <= 1e-5
            checked += 1
        else:
            assert pix == -1
    assert checked > 3000


def test_identity_camera_closed_form():
    W, H = 64, 48
    cam = identity_camera(60.0)
    M, near, far = ocam.clip_matrix(cam, W, H)
    for d in (0.5, 1.0, 7.25, 1000.0):
        pix, w = orast.project_point(M, near, far, W, H, 0.0, 0.0, -d)
        assert pix == (H // 2) * W + W // 2
        assert w == np.float32(d)
    # a point up and to the right lands in the upper-right quadrant
    pix, _ = orast.project_point(M, near, far, W, H, 0.2, 0.1, -1.0)
    assert pix // W < H // 2 and pix % W > W // 2


def test_near_far_inclusive():
    W, H = 16, 16
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    assert orast.project_point(M, near, far, W, H, 0.0, 0.0, -near)[0] >= 0
    below = np.nextafter(near, np.float32(0))
    assert orast.project_point(M, near, far, W, H, 0.0, 0.0, -below)[0] == -1
    assert orast.project_point(M, near, far, W, H, 0.0, 0.0, -far)[0] >= 0
    above = np.nextafter(far, np.float32(np.inf))
    assert orast.project_point(M, near, far, W, H, 0.0, 0.0, -above)[0] == -1


def test_screen_borders():
    """sx == W and sy == H are outside; sx == 0 and sy == 0 are inside."""
    W, H = 20, 10
    M, near, far = ocam.clip_matrix(identity_camera(70.0), W, H)
    m0, m1 = M[0], M[5]
    # choose w = M00 so that cx / w == 1 exactly
    assert orast.project_point(M, near, far, W, H, 1.0, 0.0, -m0)[0] == -1
    p, _ = orast.project_point(M, near, far, W, H, -1.0, 0.0, -m0)
    assert p >= 0 and p % W == 0
    p, _ = orast.project_point(M, near, far, W, H, np.nextafter(np.float32(1), np.float32(0)), 0.0, -m0)
    assert p % W == W - 1
    p, _ = orast.project_point(M, near, far, W, H, 0.0, 1.0, -m1)
    assert p >= 0 and p // W == 0
    assert orast.project_point(M, near, far, W, H, 0.0, -1.0, -m1)[0] == -1


def test_non_finite_and_behind_are_culled():
    W, H = 32, 32
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    bad = [(np.nan, 0, -1), (0, np.nan, -1), (0, 0, np.nan), (np.inf, 0, -1), (0, -np.inf, -1),
           (0, 0, -np.inf), (0, 0, np.inf), (0, 0, 2.0), (0.0, 0.0, 0.0)]
    for p in bad:
        assert orast.project_point(M, near, far, W, H, *p)[0] == -1
    x = np.array([b[0] for b in bad], np.float32)
    y = np.array([b[1] for b in bad], np.float32)
    z = np.array([b[2] for b in bad], np.float32)
    assert (orast.render(x, y, z, M, near, far, W, H) == EMPTY).all()


def test_empty_input():
    W, H = 8, 6
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    e = np.zeros(0, np.float32)
    keys = orast.render(e, e, e, M, near, far, W, H)
    assert keys.shape == (W * H,) and (keys == EMPTY).all()
    out = orast.resolve(keys, W, H, e, e, e, M, [e.copy()], lut=scenes.colour_lut(), lut_attr=0,
                        vel_attr=-1)
    assert (out["depth"] == 0).all() and (out["attrs"] == 0).all() and (out["rgb"] == 0).all()


def test_ties_go_to_lowest_index():
    W, H = 16, 16
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    n = 50
    x = np.full(n, 0.01, np.float32)
    y = np.full(n, 0.02, np.float32)
    z = np.full(n, -3.0, np.float32)
    z[:7] = -4.0  # farther
    keys = orast.render(x, y, z, M, near, far, W, H)
    hit = keys[keys != EMPTY]
    assert hit.size == 1 and int(hit[0]) & 0xFFFFFFFF == 7


def test_permutation_invariance():
    sc = scenes.unit_cube(n=30000, seed=11, W=96, H=64)
    M, near, far = ocam.clip_matrix(sc.cameras[0], sc.W, sc.H)
    rng = np.random.default_rng(3)
    perm = rng.permutation(sc.n)
    k0 = orast.render(sc.x, sc.y, sc.z, M, near, far, sc.W, sc.H)
    k1 = orast.render(sc.x[perm], sc.y[perm], sc.z[perm], M, near, far, sc.W, sc.H)
    assert ((k0 == EMPTY) == (k1 == EMPTY)).all()
    m = k0 != EMPTY
    # depth identical; winning point identical unless two points tie in depth
    assert ((k0[m] >> np.uint64(32)) == (k1[m] >> np.uint64(32))).all()
    i0 = (k0[m] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    i1 = perm[(k1[m] & np.uint64(0xFFFFFFFF)).astype(np.int64)]
    same = i0 == i1
    assert same.mean() > 0.999
    # where they differ, both points have exactly the same depth
    wd = lambda i: project_np(sc.x[i], sc.y[i], sc.z[i], M, near, far, sc.W, sc.H)[1]
    assert (wd(i0[~same]) == wd(i1[~same])).all()


def test_invariants_unit_cube():
    """Every covered pixel holds the minimum depth among the points that land
    there, culled points never win, every surviving point's pixel is covered by
    a key no larger than its own."""
    sc = scenes.unit_cube(n=200000, seed=0, W=128, H=128)
    M, near, far = ocam.clip_matrix(sc.cameras[0], sc.W, sc.H)
    keys = orast.render(sc.x, sc.y, sc.z, M, near, far, sc.W, sc.H)
    pix, w = project_np(sc.x, sc.y, sc.z, M, near, far, sc.W, sc.H)
    surv = pix >= 0
    own = (w.view(np.uint32).astype(np.uint64) << np.uint64(32)) | np.arange(sc.n, dtype=np.uint64)
    assert (keys[pix[surv]] <= own[surv]).all()
    winners = (keys[keys != EMPTY] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    assert surv[winners].all()
    assert (keys[pix[winners]] == own[winners]).all()
    covered = np.zeros(sc.W * sc.H, bool)
    covered[pix[surv]] = True
    assert (covered == (keys != EMPTY)).all()


def test_resolve_conversions_match_numpy():
    W, H = 8, 8
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    halfs = np.array([0.0, -0.0, 1.0, -2.5, 65504.0, 2.0 ** -24, -(2.0 ** -20), np.inf, -np.inf, np.nan,
                      0.333, 1e-5], np.float16)
    n = halfs.size
    # one point per pixel along the first rows
    xs = ((np.arange(n) % W) + 0.5) / W * 2 - 1
    ys = 1 - ((np.arange(n) // W) + 0.5) / H * 2
    tan = math.tan(math.radians(45))
    x = (xs * tan).astype(np.float32)
    y = (ys * tan).astype(np.float32)
    z = np.full(n, -1.0, np.float32)
    u8 = (np.arange(n) * 23 % 256).astype(np.uint8)
    u8[0] = 255
    u16 = (np.arange(n) * 5003 % 65536).astype(np.uint16)
    u16[1] = 65535
    f32 = np.linspace(-3, 3, n).astype(np.float32)
    keys = orast.render(x, y, z, M, near, far, W, H)
    assert (keys != EMPTY).sum() == n
    out = orast.resolve(keys, W, H, x, y, z, M, [u8, u16, halfs, f32])
    idx = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    m = keys != EMPTY
    for c, src in enumerate([u8, u16, halfs, f32]):
        ref = src.astype(np.float32)[idx[m]]
        got = out["attrs"][c][m]
        np.testing.assert_array_equal(got.view(np.uint32), ref.view(np.uint32))
        assert (out["attrs"][c][~m] == 0).all()


def test_half_signalling_nan_is_quieted():
    W, H = 4, 4
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    h = np.array([0x7C01, 0xFD55], np.uint16).view(np.float16)  # signalling NaNs (+, -)
    x = np.array([0.0, -0.6], np.float32)
    y = np.array([0.0, 0.6], np.float32)
    z = np.array([-1.0, -1.0], np.float32)
    keys = orast.render(x, y, z, M, near, far, W, H)
    out = orast.resolve(keys, W, H, x, y, z, M, [h])
    idx = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    got = {int(idx[p]): int(out["attrs"][0][p].view(np.uint32)) for p in np.nonzero(keys != EMPTY)[0]}
    assert got[0] == 0x7FC00000 | (0x001 << 13)
    assert got[1] == 0xFFC00000 | (0x155 << 13)


def ndc64(Md, p):
    c = Md @ np.append(p, 1.0)
    return c[0] / c[3], c[1] / c[3]


def test_vel2d_matches_fp64_derivative():
    """v' is the derivative of the normalised device coordinates along v:
    compare against an FP64 central difference; theta and |v'| against
    numpy's arctan2 and hypot."""
    sc = scenes.unit_cube(n=20000, seed=5, W=80, H=60)
    cam = scenes.Camera(eye=(2.0, 1.8, 1.6), target=(0.5, 0.5, 0.5), up=(0.3, -0.4, 1.0))
    M, near, far = ocam.clip_matrix(cam, sc.W, sc.H)
    assert min(abs(M[2]), abs(M[6]), abs(M[14])) > 0.05
    keys = orast.render(sc.x, sc.y, sc.z, M, near, far, sc.W, sc.H)
    out = orast.resolve(keys, sc.W, sc.H, sc.x, sc.y, sc.z, M, sc.attrs, vel_attr=0)
    v2 = out["vel2d"]
    Md = M.astype(np.float64).reshape(4, 4)
    m = np.nonzero(keys != EMPTY)[0]
    assert m.size > 500
    for p in m[::7]:
        i = int(keys[p]) & 0xFFFFFFFF
        P = np.array([sc.x[i], sc.y[i], sc.z[i]], np.float64)
        V = np.array([sc.attrs[0][i], sc.attrs[1][i], sc.attrs[2][i]], np.float64)
        h = 1e-6
        a = ndc64(Md, P + h * V)
        b = ndc64(Md, P - h * V)
        d = ((a[0] - b[0]) / (2 * h), (a[1] - b[1]) / (2 * h))
        scale = max(1.0, abs(d[0]), abs(d[1]))
        assert abs(v2[0][p] - d[0]) <= 2e-4 * scale
        assert abs(v2[1][p] - d[1]) <= 2e-4 * scale
        assert abs(v2[3][p] - math.hypot(v2[0][p], v2[1][p])) <= 1e-6 * max(1.0, v2[3][p])
        th = math.atan2(float(v2[1][p]), float(v2[0][p])) / math.pi
        assert abs(v2[2][p] - th) <= 4e-7
    empty = keys == EMPTY
    assert (v2[:, empty] == 0).all()


def test_lut_binning():
    """Bin q = floor((s - s_min) * inv_range * 256) clamped to [0, 255]."""
    W, H = 8, 1
    M, near, far = ocam.clip_matrix(identity_camera(), W, H)
    lut = scenes.colour_lut()
    s = np.array([-5.0, 0.0, 0.5 / 256, 1.5 / 256, 0.5, 255.5 / 256, 1.0, 7.0], np.float32)
    # one point per pixel of the single row
    x = (((np.arange(W) + 0.5) / W * 2 - 1) * math.tan(math.radians(45)) * (W / H)).astype(np.float32)
    y = np.zeros(W, np.float32)
    z = np.full(W, -1.0, np.float32)
    keys = orast.render(x, y, z, M, near, far, W, H)
    assert (keys != EMPTY).all()
    out = orast.resolve(keys, W, H, x, y, z, M, [s], lut=lut, lut_attr=0, lut_min=0.0, lut_inv_range=1.0)
    idx = (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)
    want_q = {0: 0, 1: 0, 2: 0, 3: 1, 4: 128, 5: 255, 6: 255, 7: 255}
    for p in range(W):
        q = want_q[int(idx[p])]
        np.testing.assert_array_equal(out["rgb"][:, p], lut[q])


def test_resolve_rgb8_colour_is_value_over_255():
    """RGB8 colour mode: each of the three uint8 attributes of the winner
    becomes (nearly) its value / 255: within one fp32 rounding of the exact
    quotient, 0 stays 0, and the ramp is monotone; empty pixels are 0."""
    W, H = 4, 4
    M, near, far = ocam.clip_matrix(scenes.Camera(eye=(0, 0, 0), target=(0, 0, -1), up=(0, 1, 0),
                                                  fovy_deg=90.0), W, H)
    vals = np.arange(256, dtype=np.uint8)
    # one point per pixel of the top-left 2x2 block is enough to check the
    # mapping; every value goes through the resolve on its own pixel
    got = np.empty((3, 256), np.float64)
    for start in range(0, 256, 4):
        v = vals[start:start + 4]
        x = np.array([-0.75, -0.25, -0.75, -0.25], np.float32)
        y = np.array([0.75, 0.75, 0.25, 0.25], np.float32)
        z = np.full(4, -1.0, np.float32)
        keys = orast.render(x, y, z, M, near, far, W, H)
        r, g, b = v.copy(), v[::-1].copy(), np.full(4, 255 - start // 4, np.uint8)
        out = orast.resolve(keys, W, H, x, y, z, M, [r, g, b], rgb_mode=1, lut_attr=0)
        rgb = out["rgb"].reshape(3, H, W)
        assert (out["rgb"][:, keys == orast.EMPTY] == 0).all()
        got[0, start:start + 4] = [rgb[0, 0, 0], rgb[0, 0, 1], rgb[0, 1, 0], rgb[0, 1, 1]]
        np.testing.assert_array_equal(rgb[1, :2, :2].ravel(), rgb[0, :2, :2].ravel()[::-1])
        assert np.all(rgb[2, :2, :2] == rgb[2, 0, 0])
    exact = vals / 255.0
    assert got[0, 0] == 0.0
    assert np.all(np.abs(got[0] - exact) <= 2.0 ** -23 * exact + 1e-45)
    assert np.all(np.diff(got[0]) > 0)


@pytest.mark.parametrize("threads", [1, 2, 3, 8, 13])
def test_multithreaded_oracle_is_bit_identical(threads):
    """The all-cores form (private key buffers merged by elementwise minimum)
    returns the single-threaded keys bit for bit, also with ties and shared
    pixels across the threads' ranges."""
    sc = scenes.unit_cube(n=200_003, seed=9, W=97, H=61)
    q = np.float32(1 / 64)
    x, y, z = ((np.floor(a / q) * q).astype(np.float32) for a in (sc.x, sc.y, sc.z))
    cam = scenes.Camera(eye=(1.6, 1.4, 1.2), target=(0.5, 0.5, 0.5))
    M, near, far = ocam.clip_matrix(cam, sc.W, sc.H)
    want = orast.render(x, y, z, M, near, far, sc.W, sc.H)
    got = orast.render_mt(x, y, z, M, near, far, sc.W, sc.H, threads)
    assert (want != orast.EMPTY).sum() > 1000
    np.testing.assert_array_equal(got, want)
