"""World splat radius of each point: mean distance to its four nearest
neighbours -- TEST INFRASTRUCTURE ONLY: tests, smoke() and the benchmark's
CPU baseline may call it; the library never does.

The paper sets the splat radius of the terrain points (its hole filling) to
the average distance between a point and its four nearest neighbours
(Sec. 4.2) and lets the rasterizer project it per pixel (Sec. 3.2).  Reading
of the arithmetic (fp32, each operation rounded in the order written):

  d(i, j) = sqrt(((x_j - x_i)^2 + (y_j - y_i)^2) + (z_j - z_i)^2)
  r_i     = (((d_1 + d_2) + d_3) + d_4) * 0.25   with d_1 <= d_2 <= d_3 <= d_4
            the four smallest d(i, j) over the other points j (j != i, every
            coordinate finite; duplicates of i count, at distance 0);
  with m < 4 such points the m smallest are summed the same way and divided
  by m; r_i = 0 when m = 0 or when a coordinate of i is not finite.

Brute force over every pair, numpy float32; np.partition and np.sort are the
only library primitives.
"""
from __future__ import annotations

import numpy as np

K = 4


def radius(x, y, z, queries=None, chunk=256):
    """r_i for i in `queries` (default: every point), float32."""
    x, y, z = (np.asarray(a, np.float32) for a in (x, y, z))
    n = x.shape[0]
    ok = np.isfinite(x) & np.isfinite(y) & np.isfinite(z)
    q = np.arange(n) if queries is None else np.asarray(queries, np.int64)
    out = np.zeros(q.shape[0], np.float32)
    xs, ys, zs = x[ok], y[ok], z[ok]
    idx = np.nonzero(ok)[0]
    chunk = max(1, min(chunk, (1 << 25) // max(1, xs.shape[0])))  # bounded temporaries
    for c0 in range(0, q.shape[0], chunk):
        qi = q[c0:c0 + chunk]
        with np.errstate(invalid="ignore", over="ignore"):
            dx = (xs[None, :] - x[qi, None]).astype(np.float32)
            dy = (ys[None, :] - y[qi, None]).astype(np.float32)
            dz = (zs[None, :] - z[qi, None]).astype(np.float32)
            d2 = ((dx * dx).astype(np.float32) + (dy * dy).astype(np.float32)).astype(np.float32)
            d2 = (d2 + (dz * dz).astype(np.float32)).astype(np.float32)
            d = np.sqrt(d2).astype(np.float32)
        d[idx[None, :] == qi[:, None]] = np.inf  # not its own neighbour
        m = min(K, xs.shape[0] - 1) if xs.shape[0] > 0 else 0
        for r, i in enumerate(qi):
            if not ok[i] or m <= 0:
                continue
            nearest = np.sort(np.partition(d[r], m - 1)[:m])
            s = np.float32(0.0)
            for v in nearest:
                s = np.float32(s + v)
            out[c0 + r] = np.float32(s * np.float32(0.25)) if m == K else np.float32(s / np.float32(m))
    return out
