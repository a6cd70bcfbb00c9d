"""Spatial layout of a point cloud (Morton order + per-batch bounding boxes)
-- TEST INFRASTRUCTURE ONLY: tests, smoke() and the benchmark's CPU baseline
may call it; the library never does.

Compute rasterization, which the multi-attribute rasterizer extends (Sec. 3.2),
stores the points sorted along a Morton (Z-order) curve in batches, so that
a batch is a compact piece of space whose bounding box can be culled as a
whole (Sec. 4.3 names the Morton-ordered data of that renderer).  The paper
gives no formula for the curve; the definition used here (a reading):

  bounding box of the finite points: lo_a = min a, hi_a = max a per axis a;
  scale_a = fp32(1024) / fp32(hi_a - lo_a)  (0 when hi_a == lo_a);
  t = fp32(fp32(a - lo_a) * scale_a)  (each operation rounded to fp32);
  q_a = 0 if not t > 0, 1023 if t >= 1023, else floor(t);
  code = sum over bits k < 10 of  bit k of q_x << 3k | bit k of q_y << (3k+1)
                                  | bit k of q_z << (3k+2);
  a point with a non-finite coordinate gets code 2^30 (after every finite one).

The layout is the stable sort of the points by code (equal codes keep the
original index order), i.e. perm[j] = original index of the j-th point, and
for each batch of B consecutive points of the sorted order the box
[min, max] per axis over its finite points (+inf / -inf when it has none).
The render's depth sample is every 8th point of that order (depth_sample).
Plain numpy, one step at a time; a stable argsort is the only library
primitive.
"""
from __future__ import annotations

import numpy as np

BITS = 10
NONFINITE_CODE = 1 << (3 * BITS)


def bbox(x, y, z):
    """(lo[3], hi[3]) float32 over the points whose three coordinates are finite."""
    x, y, z = (np.asarray(a, np.float32) for a in (x, y, z))
    ok = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    if not ok.any():
        return np.zeros(3, np.float32), np.zeros(3, np.float32)
    lo = np.array([a[ok].min() for a in (x, y, z)], np.float32)
    hi = np.array([a[ok].max() for a in (x, y, z)], np.float32)
    return lo, hi


def quantise(a, lo, hi):
    """Cell index in [0, 1023] along one axis (fp32 arithmetic as defined above)."""
    a = np.asarray(a, np.float32)
    lo, hi = np.float32(lo), np.float32(hi)
    ext = np.float32(hi - lo)
    scale = np.float32(np.float32(1 << BITS) / ext) if ext > 0 else np.float32(0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        t = (a - lo).astype(np.float32)
        t = (t * scale).astype(np.float32)
        q = np.where(~(t > 0), 0, np.where(t >= np.float32((1 << BITS) - 1), (1 << BITS) - 1,
                                           np.floor(np.where(t > 0, t, 0)).astype(np.int64)))
    return q.astype(np.int64)


def interleave(qx, qy, qz):
    """Bit k of qx, qy, qz to bits 3k, 3k+1, 3k+2 of the code."""
    code = np.zeros(np.shape(qx), np.int64)
    for k in range(BITS):
        code |= ((np.asarray(qx) >> k) & 1) << (3 * k)
        code |= ((np.asarray(qy) >> k) & 1) << (3 * k + 1)
        code |= ((np.asarray(qz) >> k) & 1) << (3 * k + 2)
    return code


def morton_codes(x, y, z):
    x, y, z = (np.asarray(a, np.float32) for a in (x, y, z))
    lo, hi = bbox(x, y, z)
    code = interleave(quantise(x, lo[0], hi[0]), quantise(y, lo[1], hi[1]), quantise(z, lo[2], hi[2]))
    ok = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    return np.where(ok, code, NONFINITE_CODE)


def layout(x, y, z, batch=2048):
    """(perm uint32[n], boxes float32[nbatch][2][3]) of the Morton layout."""
    x, y, z = (np.asarray(a, np.float32) for a in (x, y, z))
    perm = np.argsort(morton_codes(x, y, z), kind="stable").astype(np.uint32)
    n = x.shape[0]
    nb = (n + batch - 1) // batch
    boxes = np.empty((nb, 2, 3), np.float32)
    for b in range(nb):
        idx = perm[b * batch:(b + 1) * batch]
        px, py, pz = x[idx], y[idx], z[idx]
        ok = np.isfinite(px) & np.isfinite(py) & np.isfinite(pz)
        for a, v in enumerate((px, py, pz)):
            boxes[b, 0, a] = v[ok].min() if ok.any() else np.float32(np.inf)
            boxes[b, 1, a] = v[ok].max() if ok.any() else np.float32(-np.inf)
    return perm, boxes


def depth_sample(x, y, z, perm, batch=2048):
    """The render's depth sample of a layout (a reading of how to spread the
    first-drawn points evenly over the cloud): every 8th point of the layout
    order, positions 0, 8, 16, ...  Returns (original indices uint32
    [ceil(n / 8)], boxes of its consecutive batches of `batch` sample points,
    as layout() gives them)."""
    x, y, z = (np.asarray(a, np.float32) for a in (x, y, z))
    sidx = np.asarray(perm, np.uint32)[0::8]
    ns = sidx.shape[0]
    nb = (ns + batch - 1) // batch
    boxes = np.empty((nb, 2, 3), np.float32)
    for b in range(nb):
        idx = sidx[b * batch:(b + 1) * batch]
        px, py, pz = x[idx], y[idx], z[idx]
        ok = np.isfinite(px) & np.isfinite(py) & np.isfinite(pz)
        for a, v in enumerate((px, py, pz)):
            boxes[b, 0, a] = v[ok].min() if ok.any() else np.float32(np.inf)
            boxes[b, 1, a] = v[ok].max() if ok.any() else np.float32(-np.inf)
    return sidx, boxes
