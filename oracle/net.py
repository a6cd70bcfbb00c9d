"""FP64 CPU oracle of the post-processing network -- TEST INFRASTRUCTURE ONLY.

The paper post-processes the rasterizer's G-buffers with a U-Net (Sec. 3.3):
an encoder of convolution blocks with 2x2 average pooling between levels and
a decoder that upsamples and fuses skip connections, trained with a
reconstruction loss plus a 2D total-variation term (Eq. 1) by Adam (lr 1e-3).
This oracle computes the small encoder-decoder this build trains instead
(the paper's own gated-conv variant is not built):

  input 8 channels (RGB, depth, Vel2D) at H x W (H, W multiples of 8)
  level 1:  conv3x3 8->32, ReLU, conv3x3 32->32, ReLU          -> s1
  pool 2x2 (average)
  level 2:  conv3x3 32->64, ReLU, conv3x3 64->64, ReLU         -> s2
  pool
  level 3:  conv3x3 64->128, ReLU, conv3x3 128->128, ReLU      -> s3
  pool
  level 4:  conv3x3 128->256, ReLU, conv3x3 256->256, ReLU
  up x2 (bilinear), concat [up, s3] (384): conv 384->128, ReLU, conv 128->128, ReLU
  up x2, concat [up, s2] (192):            conv 192->64,  ReLU, conv 64->64,   ReLU
  up x2, concat [up, s1] (96):             conv 96->32,   ReLU, conv 32->32,   ReLU
  head: conv1x1 32->3 (linear)

Conventions (readings where the paper is silent): 3x3 convolutions use zero
padding 1 and a bias; bilinear upsampling samples the source at
(o + 0.5)/2 - 0.5 clamped to the edge (half-pixel centres); the loss is the
mean squared error over all outputs plus lambda * (mean |horizontal
difference| + mean |vertical difference|) of the output; Adam uses
beta = (0.9, 0.999), eps = 1e-8 and bias correction.

Everything is plain numpy float64 in NCHW layout, one operation at a time; a
matrix product is the only library primitive.
"""
from __future__ import annotations

import numpy as np

IN_CH, OUT_CH = 8, 3
WIDTHS = (32, 64, 128, 256)

# (name, in channels, out channels, kernel size) in forward order
LAYERS = [
    ("e1a", 8, 32, 3), ("e1b", 32, 32, 3),
    ("e2a", 32, 64, 3), ("e2b", 64, 64, 3),
    ("e3a", 64, 128, 3), ("e3b", 128, 128, 3),
    ("e4a", 128, 256, 3), ("e4b", 256, 256, 3),
    ("d3a", 384, 128, 3), ("d3b", 128, 128, 3),
    ("d2a", 192, 64, 3), ("d2b", 64, 64, 3),
    ("d1a", 96, 32, 3), ("d1b", 32, 32, 3),
    ("head", 32, 3, 1),
]


def layer_table(widths=WIDTHS, in_ch=IN_CH, out_ch=OUT_CH):
    """LAYERS for other channel widths (small networks for gradient checks)."""
    a, b, c, d = widths
    return [("e1a", in_ch, a, 3), ("e1b", a, a, 3), ("e2a", a, b, 3), ("e2b", b, b, 3),
            ("e3a", b, c, 3), ("e3b", c, c, 3), ("e4a", c, d, 3), ("e4b", d, d, 3),
            ("d3a", d + c, c, 3), ("d3b", c, c, 3), ("d2a", c + b, b, 3), ("d2b", b, b, 3),
            ("d1a", b + a, a, 3), ("d1b", a, a, 3), ("head", a, out_ch, 1)]


def features(planes):
    """Network input from G-buffer planes [N, 8, H, W] (r, g, b, depth, v'x, v'y,
    theta, |v'|): the depth plane becomes inverse depth, 0 where no point."""
    x = np.array(planes, dtype=np.float64, copy=True)
    d = x[:, 3]
    x[:, 3] = np.where(d > 0, 1.0 / np.where(d > 0, d, 1.0), 0.0)
    return x


def to_blob(P, table=None):
    """Parameters as one flat float64 vector: per layer W [Co, Ci, k, k] then b."""
    table = table or LAYERS
    return np.concatenate([np.concatenate([P[n][0].reshape(-1), P[n][1]]) for n, *_ in table])


def from_blob(blob, table=None):
    table = table or LAYERS
    P, o = {}, 0
    for name, ci, co, k in table:
        nw = co * ci * k * k
        P[name] = (np.asarray(blob[o:o + nw], np.float64).reshape(co, ci, k, k), np.asarray(blob[o + nw:o + nw + co], np.float64))
        o += nw + co
    return P


def init_params(rng, table=None):
    """He-normal weights, zero biases: {name: (W [Co, Ci, k, k], b [Co])}."""
    table = table or LAYERS
    P = {}
    for name, ci, co, k in table:
        std = np.sqrt(2.0 / (ci * k * k))
        P[name] = (rng.standard_normal((co, ci, k, k)) * std, np.zeros(co))
    return P


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------

def _im2col3(x):
    """[N, C, H, W] -> [N, C*9, H*W]; row c*9 + ky*3 + kx holds x[c, y+ky-1, x+kx-1] (zero outside)."""
    N, C, H, W = x.shape
    xp = np.zeros((N, C, H + 2, W + 2))
    xp[:, :, 1:-1, 1:-1] = x
    cols = np.empty((N, C, 9, H, W))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, ky * 3 + kx] = xp[:, :, ky:ky + H, kx:kx + W]
    return cols.reshape(N, C * 9, H * W)


def _col2im3(cols, shape):
    """Adjoint of _im2col3."""
    N, C, H, W = shape
    cols = cols.reshape(N, C, 9, H, W)
    xp = np.zeros((N, C, H + 2, W + 2))
    for ky in range(3):
        for kx in range(3):
            xp[:, :, ky:ky + H, kx:kx + W] += cols[:, :, ky * 3 + kx]
    return xp[:, :, 1:-1, 1:-1]


def conv(x, Wt, b):
    """Cross-correlation with zero padding (k // 2) and bias; k in {1, 3}."""
    N, C, H, Wd = x.shape
    co, ci, k, _ = Wt.shape
    assert ci == C
    cols = _im2col3(x) if k == 3 else x.reshape(N, C, H * Wd)
    y = np.matmul(Wt.reshape(co, ci * k * k), cols) + b[None, :, None]
    return y.reshape(N, co, H, Wd), cols


def conv_backward(dy, cols, Wt, xshape):
    N, co, H, Wd = dy.shape
    k = Wt.shape[2]
    dy2 = dy.reshape(N, co, H * Wd)
    Wm = Wt.reshape(co, -1)
    dW = np.matmul(dy2, cols.transpose(0, 2, 1)).sum(axis=0).reshape(Wt.shape)
    db = dy2.sum(axis=(0, 2))
    dcols = np.matmul(Wm.T, dy2)
    dx = _col2im3(dcols, xshape) if k == 3 else dcols.reshape(xshape)
    return dx, dW, db


def relu(x):
    return np.maximum(x, 0.0)


def avgpool2(x):
    N, C, H, W = x.shape
    return x.reshape(N, C, H // 2, 2, W // 2, 2).mean(axis=(3, 5))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=2), 2, axis=3) / 4.0


def upsample_matrix(n):
    """[2n, n] bilinear x2 interpolation with half-pixel centres, edge-clamped."""
    U = np.zeros((2 * n, n))
    for o in range(2 * n):
        src = max((o + 0.5) / 2.0 - 0.5, 0.0)
        i0 = min(int(np.floor(src)), n - 1)
        i1 = min(i0 + 1, n - 1)
        f = src - i0
        U[o, i0] += 1.0 - f
        U[o, i1] += f
    return U


def upsample2(x):
    """y[n, c] = Uh @ x[n, c] @ Uw^T (rows, then columns interpolated)."""
    N, C, H, W = x.shape
    Uh, Uw = upsample_matrix(H), upsample_matrix(W)
    return np.matmul(Uh, np.matmul(x, Uw.T))


def upsample2_backward(dy):
    """Adjoint of upsample2: dx[n, c] = Uh^T @ dy[n, c] @ Uw."""
    N, C, H2, W2 = dy.shape
    Uh, Uw = upsample_matrix(H2 // 2), upsample_matrix(W2 // 2)
    return np.matmul(Uh.T, np.matmul(dy, Uw))


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def forward(P, x):
    """Returns (output [N, 3, H, W], cache for backward)."""
    cache = {}

    def cv(name, inp, act=True):
        Wt, b = P[name]
        z, cols = conv(inp, Wt, b)
        cache[name] = (inp.shape, cols, z)
        return relu(z) if act else z

    s1 = cv("e1b", cv("e1a", x))
    s2 = cv("e2b", cv("e2a", avgpool2(s1)))
    s3 = cv("e3b", cv("e3a", avgpool2(s2)))
    s4 = cv("e4b", cv("e4a", avgpool2(s3)))
    d3 = cv("d3b", cv("d3a", np.concatenate([upsample2(s4), s3], axis=1)))
    d2 = cv("d2b", cv("d2a", np.concatenate([upsample2(d3), s2], axis=1)))
    d1 = cv("d1b", cv("d1a", np.concatenate([upsample2(d2), s1], axis=1)))
    y = cv("head", d1, act=False)
    cache["chans"] = (s1.shape[1], s2.shape[1], s3.shape[1], s4.shape[1], d3.shape[1], d2.shape[1])
    return y, cache


def backward(P, cache, dy):
    """Gradients {name: (dW, db)} of sum(dy * output)."""
    G = {}

    def bw(name, g, act=True):
        shape, cols, z = cache[name]
        if act:
            g = g * (z > 0)
        dx, dW, db = conv_backward(g, cols, P[name][0], shape)
        G[name] = (dW, db)
        return dx

    c1, c2, c3, c4, cd3, cd2 = cache["chans"]
    g = bw("head", dy, act=False)
    g = bw("d1a", bw("d1b", g))
    g_up, g_s1 = g[:, :cd2], g[:, cd2:]
    g = bw("d2a", bw("d2b", upsample2_backward(g_up)))
    g_up, g_s2 = g[:, :cd3], g[:, cd3:]
    g = bw("d3a", bw("d3b", upsample2_backward(g_up)))
    g_up, g_s3 = g[:, :c4], g[:, c4:]
    g = bw("e4a", bw("e4b", upsample2_backward(g_up)))
    g = bw("e3a", bw("e3b", avgpool2_backward(g) + g_s3))
    g = bw("e2a", bw("e2b", avgpool2_backward(g) + g_s2))
    bw("e1a", bw("e1b", avgpool2_backward(g) + g_s1))
    return G


def loss(y, t, lam_tv=1e-3):
    """(loss, dloss/dy): mean squared error + lam_tv * (mean|dx| + mean|dy|) of y."""
    d = y - t
    L = np.mean(d * d)
    g = 2.0 * d / d.size
    if lam_tv:
        hx = y[..., :, 1:] - y[..., :, :-1]
        hy = y[..., 1:, :] - y[..., :-1, :]
        L += lam_tv * (np.mean(np.abs(hx)) + np.mean(np.abs(hy)))
        sx = np.sign(hx) * lam_tv / hx.size
        sy = np.sign(hy) * lam_tv / hy.size
        g[..., :, 1:] += sx
        g[..., :, :-1] -= sx
        g[..., 1:, :] += sy
        g[..., :-1, :] -= sy
    return L, g


def adam(P, G, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; state = {"t": int, name: (mW, vW, mb, vb)}.  Returns new params."""
    t = state.get("t", 0) + 1
    state["t"] = t
    out = {}
    for name, (Wt, b) in P.items():
        dW, db = G[name]
        mW, vW, mb, vb = state.get(name, (0.0, 0.0, 0.0, 0.0))
        mW = b1 * mW + (1 - b1) * dW
        vW = b2 * vW + (1 - b2) * dW * dW
        mb = b1 * mb + (1 - b1) * db
        vb = b2 * vb + (1 - b2) * db * db
        state[name] = (mW, vW, mb, vb)
        c1, c2 = 1 - b1 ** t, 1 - b2 ** t
        out[name] = (Wt - lr * (mW / c1) / (np.sqrt(vW / c2) + eps), b - lr * (mb / c1) / (np.sqrt(vb / c2) + eps))
    return out


def psnr(a, b):
    """10 log10(1 / MSE) for images in [0, 1]."""
    mse = float(np.mean((np.asarray(a, np.float64) - np.asarray(b, np.float64)) ** 2))
    return float("inf") if mse == 0 else 10.0 * np.log10(1.0 / mse)
