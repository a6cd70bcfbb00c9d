"""Pins of the paper-network oracle (oracle/unet.py) against torch's CPU
float64 routines (conv2d, conv_transpose2d, elu, sigmoid, avg_pool2d and
autograd: an independent implementation), and against central finite
differences of the loss."""
import numpy as np
import pytest

from oracle import net as onet
from oracle import unet as ounet

torch = pytest.importorskip("torch")
F = torch.nn.functional

SMALL = (4, 8, 8, 16, 16)


def torch_forward(P, x):
    t = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    TP = {k: (t(w), t(b)) for k, (w, b) in P.items()}
    x = torch.tensor(x, dtype=torch.float64)
    Wd, bd = TP["desc"]
    d = [F.conv2d(x, Wd[:, :, None, None], bd)]
    for _ in range(4):
        d.append(F.avg_pool2d(d[-1], 2))
    gate = lambda z: F.elu(z[:, :z.shape[1] // 2]) * torch.sigmoid(z[:, z.shape[1] // 2:])
    ys, inp = [], x
    for l in range(5):
        W, b = TP[f"enc{l}"]
        y = gate(F.conv2d(torch.cat([inp, d[l]], 1), W, b, padding=1))
        ys.append(y)
        inp = F.avg_pool2d(y, 2)
    up_in = ys[4]
    for l in (3, 2, 1, 0):
        T, bt = TP[f"up{l}"]
        u = F.conv_transpose2d(up_in, T.permute(3, 2, 0, 1), bt, stride=2)
        W, b = TP[f"dec{l}"]
        up_in = gate(F.conv2d(torch.cat([u, ys[l]], 1), W, b, padding=1))
    Wh, bh = TP["head"]
    return F.conv2d(up_in, Wh[:, :, None, None], bh), TP


def test_forward_and_backward_match_torch():
    rng = np.random.default_rng(0)
    P = ounet.init_params(rng, SMALL)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((2, 8, 32, 48))
    y, cache = ounet.forward(P, x)
    ty, TP = torch_forward(P, x)
    assert np.max(np.abs(y - ty.detach().numpy())) < 1e-11
    dy = rng.standard_normal(y.shape)
    G = ounet.backward(P, cache, dy)
    (ty * torch.tensor(dy)).sum().backward()
    for k, (tw, tb) in TP.items():
        gw, gb = G[k]
        assert np.max(np.abs(gw - tw.grad.numpy())) <= 1e-10 * (1 + np.abs(gw).max()), k
        assert np.max(np.abs(gb - tb.grad.numpy())) <= 1e-10 * (1 + np.abs(gb).max()), k


def test_gradient_finite_differences():
    rng = np.random.default_rng(3)
    widths = (2, 4, 4, 4, 4)
    P = ounet.init_params(rng, widths)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((1, 8, 16, 16))
    t = rng.random((1, 3, 16, 16))

    def loss(P):
        y, _ = ounet.forward(P, x)
        return onet.loss(y, t, lam_tv=1e-3)[0]

    y, cache = ounet.forward(P, x)
    _, gy = onet.loss(y, t, lam_tv=1e-3)
    G = ounet.backward(P, cache, gy)
    for name in ("desc", "enc0", "enc4", "up3", "up0", "dec2", "head"):
        W, b = P[name]
        for idx in [tuple(rng.integers(0, s) for s in W.shape) for _ in range(3)]:
            h = 1e-6
            Wp, Wm = W.copy(), W.copy()
            Wp[idx] += h
            Wm[idx] -= h
            num = (loss({**P, name: (Wp, b)}) - loss({**P, name: (Wm, b)})) / (2 * h)
            ana = G[name][0][idx]
            assert abs(num - ana) <= 1e-6 * max(1e-3, abs(num)) + 1e-9, (name, idx, num, ana)


def test_blob_roundtrip_and_count():
    rng = np.random.default_rng(1)
    P = ounet.init_params(rng, SMALL)
    blob = ounet.to_blob(P, SMALL)
    assert blob.size == ounet.param_count(SMALL)
    Q = ounet.from_blob(blob, SMALL)
    assert all(np.array_equal(P[k][0], Q[k][0]) and np.array_equal(P[k][1], Q[k][1]) for k in P)
    # the paper's widths: about 27 million parameters
    assert 26_000_000 < ounet.param_count() < 29_000_000


def test_padded_inference_matches_torch():
    """Frames that are not multiples of 16: torch pads with F.pad, runs its own
    composition and crops; a frame that already is one is the plain forward."""
    rng = np.random.default_rng(11)
    P = ounet.init_params(rng, SMALL)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((1, 8, 21, 35))
    got = ounet.infer(P, x)
    assert got.shape == (1, 3, 21, 35)
    ty, _ = torch_forward(P, F.pad(torch.tensor(x), (0, 13, 0, 11)).numpy())
    assert np.max(np.abs(got - ty.detach().numpy()[:, :, :21, :35])) < 1e-11
    x16 = rng.random((1, 8, 32, 16))
    assert np.array_equal(ounet.infer(P, x16), ounet.forward(P, x16)[0])
