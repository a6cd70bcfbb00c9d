"""Pins of the Morton layout oracle (oracle/layout.py) against facts that do
not come from its own code: the bit-interleaving by the classic magic-mask
spreading and by hand-computed values, exact cell boundaries, the Z-order of
the eight octants, and the invariants of a stable sort and of bounding boxes
checked by brute force."""
import numpy as np

from oracle import layout as olay


def spread_magic(v):
    """Textbook 10-bit -> 30-bit spreading (bit k to bit 3k) by shifts and masks."""
    v = np.asarray(v, np.int64) & 0x3FF
    v = (v | (v << 16)) & 0x030000FF
    v = (v | (v << 8)) & 0x0300F00F
    v = (v | (v << 4)) & 0x030C30C3
    v = (v | (v << 2)) & 0x09249249
    return v


def test_interleave_by_hand_and_by_masks():
    assert olay.interleave(1, 0, 0) == 1
    assert olay.interleave(0, 1, 0) == 2
    assert olay.interleave(0, 0, 1) == 4
    assert olay.interleave(2, 0, 0) == 8
    assert olay.interleave(0, 0, 512) == 1 << 29
    assert olay.interleave(1023, 1023, 1023) == (1 << 30) - 1
    rng = np.random.default_rng(0)
    q = rng.integers(0, 1024, size=(3, 5000))
    want = spread_magic(q[0]) | (spread_magic(q[1]) << 1) | (spread_magic(q[2]) << 2)
    assert np.array_equal(olay.interleave(q[0], q[1], q[2]), want)


def test_quantise_cell_boundaries():
    # box [0, 1]: scale 1024 exactly, so the centre of cell k maps to k
    k = np.arange(1024)
    a = (k / 1024.0 + 1.0 / 2048.0).astype(np.float32)
    assert np.array_equal(olay.quantise(a, 0.0, 1.0), k)
    # the box ends, below/above it, and a degenerate extent
    assert olay.quantise(np.float32(0.0), 0.0, 1.0) == 0
    assert olay.quantise(np.float32(1.0), 0.0, 1.0) == 1023
    assert olay.quantise(np.float32(-5.0), 0.0, 1.0) == 0
    assert olay.quantise(np.float32(7.0), 0.0, 1.0) == 1023
    assert olay.quantise(np.float32(3.0), 3.0, 3.0) == 0


def test_octants_follow_the_z_curve():
    # the eight corners of a cube: x varies fastest, then y, then z
    c = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], np.float32)
    perm, boxes = olay.layout(c[::-1, 0].copy(), c[::-1, 1].copy(), c[::-1, 2].copy(), batch=4)
    got = c[::-1][perm]
    assert np.array_equal(got, c)
    assert np.array_equal(boxes[0], [[0, 0, 0], [1, 1, 0]])
    assert np.array_equal(boxes[1], [[0, 0, 1], [1, 1, 1]])


def test_layout_is_a_stable_sort_with_tight_boxes():
    rng = np.random.default_rng(3)
    n = 20000
    # few distinct cells, so that many codes tie; some non-finite points
    x = (rng.integers(0, 8, n) / 7.0).astype(np.float32)
    y = rng.random(n, dtype=np.float32)
    z = (rng.integers(0, 3, n) * 0.25).astype(np.float32)
    x[rng.integers(0, n, 50)] = np.nan
    y[rng.integers(0, n, 50)] = np.inf
    perm, boxes = olay.layout(x, y, z, batch=512)
    assert np.array_equal(np.sort(perm), np.arange(n))
    codes = olay.morton_codes(x, y, z)
    # brute force: sort (code, index) pairs
    want = np.array(sorted(range(n), key=lambda i: (int(codes[i]), i)), np.uint32)
    assert np.array_equal(perm, want)
    ok = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    assert not ok[perm[-int((~ok).sum()):]].any()  # non-finite points last
    for b in range(boxes.shape[0]):
        idx = perm[b * 512:(b + 1) * 512]
        idx = idx[ok[idx]]
        if idx.size == 0:
            assert np.all(np.isinf(boxes[b]))
            continue
        for a, v in enumerate((x, y, z)):
            assert boxes[b, 0, a] == v[idx].min() and boxes[b, 1, a] == v[idx].max()


def test_batches_are_compact():
    # 64k uniform points: a Morton batch of 512 spans a small part of the box
    rng = np.random.default_rng(5)
    x, y, z = rng.random((3, 65536), dtype=np.float32)
    perm, boxes = olay.layout(x, y, z, batch=512)
    ext = boxes[:, 1] - boxes[:, 0]
    assert np.median(ext.prod(axis=1)) < 4.0 / 128  # generation order: ~1


def test_depth_sample_is_every_8th_point_with_tight_boxes():
    rng = np.random.default_rng(9)
    for n in (1, 7, 8, 9, 5000, 40001):
        x, y, z = rng.random((3, n), dtype=np.float32)
        if n > 100:
            y[::97] = np.nan
        perm, _ = olay.layout(x, y, z, batch=64)
        sidx, boxes = olay.depth_sample(x, y, z, perm, batch=64)
        assert sidx.shape[0] == (n + 7) // 8
        assert all(int(sidx[j]) == int(perm[8 * j]) for j in range(sidx.shape[0]))
        assert boxes.shape[0] == (sidx.shape[0] + 63) // 64
        for b in range(boxes.shape[0]):
            idx = sidx[64 * b:64 * (b + 1)]
            ok = np.isfinite(x[idx]) & np.isfinite(y[idx]) & np.isfinite(z[idx])
            for a, v in enumerate((x, y, z)):
                vv = v[idx][ok]
                if vv.size:
                    assert boxes[b, 0, a] == vv.min() and boxes[b, 1, a] == vv.max()
                    assert np.all(vv >= boxes[b, 0, a]) and np.all(vv <= boxes[b, 1, a])
                else:
                    assert boxes[b, 0, a] == np.inf and boxes[b, 1, a] == -np.inf
