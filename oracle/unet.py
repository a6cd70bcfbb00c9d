"""FP64 CPU oracle of the paper's own post-processing network -- TEST
INFRASTRUCTURE ONLY: tests, smoke() and the benchmark's CPU baseline may call
it; the library never does.

Sec. 3.3 and Fig. 4: a U-Net whose encoder has 4 stages of downsampling with
gated convolution blocks (each gated convolution followed by ELU and 2x2
average pooling), channels growing 64-128-256-512-1024; a decoder that
upsamples with transposed convolutions and fuses the skip connections; the
G-buffers pass through a 1x1 convolution that keeps their channel count, are
downscaled to 5 resolutions (factor 0.5 each) and are concatenated to the
first blocks of the encoder at the matching resolutions.  Readings where the
paper is silent (each also in the design notes):

  gated convolution: z = conv3x3(x) with 2C outputs (zero padding 1, bias),
      y = ELU(z[:C]) * sigmoid(z[C:])  (ELU with alpha 1);
  encoder level l (l = 0..4, widths w_l): input = concat[x_l, d_l] with
      x_0 the 8 G-buffer channels (depth as 1/depth, as the small network),
      x_l = avgpool2(y_{l-1}) for l >= 1, d_l = avgpool2^l(conv1x1(x_0))
      (8 channels, bias); y_l = gate(conv(input));
  decoder level l (l = 3..0): u_l = convT2x2 stride 2 (w_{l+1} -> w_l, bias)
      of the level above (y_4, then the decoder outputs), y'_l = gate(conv(
      concat[u_l, y_l]));
  head: conv1x1(w_0 -> 3), linear;
  inference on frames that are not multiples of 16: zero-pad, run, crop.
  convT2x2: out[2i+a, 2j+b, co] = sum_ci in[i, j, ci] * T[a][b][co][ci] + bias[co].

Parameter blob (float64 here, fp32 for the library), per layer in this order:
desc (W [8][8], b [8]), enc0..enc4 (W [2 w_l][c_in][3][3], b [2 w_l]),
up3 (T [2][2][w_3][w_4], b [w_3]), dec3 (W [2 w_3][2 w_3][3][3], b [2 w_3]),
up2, dec2, up1, dec1, up0, dec0, head (W [3][w_0], b [3]).

Plain numpy float64 in NCHW layout; a matrix product is the only library
primitive (the 3x3 convolution reuses the small network oracle's).
"""
from __future__ import annotations

import numpy as np

from . import net as _net

WIDTHS = (64, 128, 256, 512, 1024)
IN_CH, DESC_CH, OUT_CH = 8, 8, 3


def layers(widths=WIDTHS):
    """[(name, kind, shape of W, channels of b)] in blob order."""
    w = widths
    L = [("desc", "conv1", (DESC_CH, IN_CH), DESC_CH)]
    cin = IN_CH
    for l in range(5):
        L.append((f"enc{l}", "gate3", (2 * w[l], cin + DESC_CH, 3, 3), 2 * w[l]))
        cin = w[l]
    for l in (3, 2, 1, 0):
        L.append((f"up{l}", "tconv", (2, 2, w[l], w[l + 1]), w[l]))
        L.append((f"dec{l}", "gate3", (2 * w[l], 2 * w[l], 3, 3), 2 * w[l]))
    L.append(("head", "conv1", (OUT_CH, w[0]), OUT_CH))
    return L


def param_count(widths=WIDTHS):
    return sum(int(np.prod(s)) + b for _, _, s, b in layers(widths))


def from_blob(blob, widths=WIDTHS):
    P, o = {}, 0
    for name, _, shape, nb in layers(widths):
        k = int(np.prod(shape))
        P[name] = (np.asarray(blob[o:o + k], np.float64).reshape(shape), np.asarray(blob[o + k:o + k + nb], np.float64))
        o += k + nb
    return P


def to_blob(P, widths=WIDTHS):
    return np.concatenate([np.concatenate([P[n][0].reshape(-1), P[n][1]]) for n, *_ in layers(widths)])


def init_params(rng, widths=WIDTHS):
    """He-normal weights (fan-in), zero biases."""
    P = {}
    for name, kind, shape, nb in layers(widths):
        if kind == "gate3":
            fan = shape[1] * 9
        elif kind == "tconv":
            fan = shape[3]
        else:
            fan = shape[1]
        P[name] = (rng.standard_normal(shape) * np.sqrt(2.0 / fan), np.zeros(nb))
    return P


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------

def elu(x):
    return np.where(x > 0, x, np.expm1(np.minimum(x, 0.0)))


def sigmoid(x):
    with np.errstate(over="ignore"):  # exp(-x) = inf for x far below 0: the value is 0, as it should be
        return 1.0 / (1.0 + np.exp(-x))


def conv1(x, Wm, b):
    """1x1 convolution, Wm [Co][Ci]."""
    N, C, H, W = x.shape
    y = np.matmul(Wm, x.reshape(N, C, H * W)) + b[None, :, None]
    return y.reshape(N, Wm.shape[0], H, W)


def tconv(x, T, b):
    """2x2 stride-2 transposed convolution, T [2][2][Co][Ci]."""
    N, C, H, W = x.shape
    Co = T.shape[2]
    y = np.empty((N, Co, 2 * H, 2 * W))
    for a in range(2):
        for c in range(2):
            y[:, :, a::2, c::2] = np.matmul(T[a, c], x.reshape(N, C, H * W)).reshape(N, Co, H, W)
    return y + b[None, :, None, None]


def tconv_backward(dy, x, T):
    N, Co, H2, W2 = dy.shape
    C = x.shape[1]
    H, W = H2 // 2, W2 // 2
    xm = x.reshape(N, C, H * W)
    dx = np.zeros((N, C, H * W))
    dT = np.zeros_like(T)
    for a in range(2):
        for c in range(2):
            g = dy[:, :, a::2, c::2].reshape(N, Co, H * W)
            dx += np.matmul(T[a, c].T, g)
            dT[a, c] = np.matmul(g, xm.transpose(0, 2, 1)).sum(axis=0)
    return dx.reshape(N, C, H, W), dT, dy.sum(axis=(0, 2, 3))


def gate(z):
    C = z.shape[1] // 2
    return elu(z[:, :C]) * sigmoid(z[:, C:])


def gate_backward(dy, z):
    C = z.shape[1] // 2
    f, g = z[:, :C], z[:, C:]
    s = sigmoid(g)
    e = elu(f)
    de = np.where(f > 0, 1.0, np.exp(np.minimum(f, 0.0)))
    return np.concatenate([dy * s * de, dy * e * s * (1.0 - s)], axis=1)


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def forward(P, x):
    """x: features [N, 8, H, W] (H, W multiples of 16).  Returns (output
    [N, 3, H, W], cache for backward)."""
    cache = {"x": x}
    d = [conv1(x, P["desc"][0], P["desc"][1])]
    for _ in range(4):
        d.append(_net.avgpool2(d[-1]))
    cache["d"] = d
    ys = []
    inp = x
    for l in range(5):
        cat = np.concatenate([inp, d[l]], axis=1)
        z, cols = _net.conv(cat, P[f"enc{l}"][0], P[f"enc{l}"][1])
        y = gate(z)
        cache[f"enc{l}"] = (cat.shape, cols, z)
        ys.append(y)
        inp = _net.avgpool2(y) if l < 4 else None
    cache["ys"] = ys
    up_in = ys[4]
    for l in (3, 2, 1, 0):
        u = tconv(up_in, P[f"up{l}"][0], P[f"up{l}"][1])
        cat = np.concatenate([u, ys[l]], axis=1)
        z, cols = _net.conv(cat, P[f"dec{l}"][0], P[f"dec{l}"][1])
        cache[f"up{l}"] = up_in
        cache[f"dec{l}"] = (cat.shape, cols, z)
        up_in = gate(z)
    cache["last"] = up_in
    out = conv1(up_in, P["head"][0], P["head"][1])
    return out, cache


def infer(P, x):
    """Inference on any H x W (a reading: the paper's frames need not be
    multiples of 16): the input zero-padded at the bottom and right to the
    next multiples of 16 (a padded pixel is an empty pixel, every channel 0),
    the top-left H x W of the output."""
    N, C, H, W = x.shape
    Hp, Wp = -(-H // 16) * 16, -(-W // 16) * 16
    xp = np.zeros((N, C, Hp, Wp))
    xp[:, :, :H, :W] = x
    return forward(P, xp)[0][:, :, :H, :W]


def backward(P, cache, dy):
    """Gradients {name: (dW, db)} of sum(dy * output)."""
    G = {}
    last = cache["last"]
    N, C0, H, W = last.shape
    Wh = P["head"][0]
    G["head"] = (np.einsum("nohw,nchw->oc", dy, last), dy.sum(axis=(0, 2, 3)))
    g = np.einsum("oc,nohw->nchw", Wh, dy)
    ys = cache["ys"]
    g_skip = {}
    # the decoder ran level 3 first and level 0 last: walk it back from level 0
    for l in (0, 1, 2, 3):
        shape, cols, z = cache[f"dec{l}"]
        dz = gate_backward(g, z)
        dcat, dW, db = _net.conv_backward(dz, cols, P[f"dec{l}"][0], shape)
        G[f"dec{l}"] = (dW, db)
        w_l = ys[l].shape[1]
        du, g_skip[l] = dcat[:, :w_l], dcat[:, w_l:]
        dx, dT, dbt = tconv_backward(du, cache[f"up{l}"], P[f"up{l}"][0])
        G[f"up{l}"] = (dT, dbt)
        g = dx  # gradient of the level above's output (y_4 for l = 3)
    # encoder, deepest first
    g_y = g
    g_d = [None] * 5
    for l in (4, 3, 2, 1, 0):
        if l < 4:
            g_y = g_y + g_skip[l]
        shape, cols, z = cache[f"enc{l}"]
        dz = gate_backward(g_y, z)
        dcat, dW, db = _net.conv_backward(dz, cols, P[f"enc{l}"][0], shape)
        G[f"enc{l}"] = (dW, db)
        cin = shape[1] - DESC_CH
        g_in, g_d[l] = dcat[:, :cin], dcat[:, cin:]
        if l > 0:
            g_y = _net.avgpool2_backward(g_in)
    # descriptors: d_l = pool^l(d_0)
    gd = g_d[4]
    for l in (3, 2, 1, 0):
        gd = _net.avgpool2_backward(gd) + g_d[l]
    x = cache["x"]
    G["desc"] = (np.einsum("nohw,nchw->oc", gd, x), gd.sum(axis=(0, 2, 3)))
    return G
