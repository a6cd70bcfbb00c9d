"""Pins for the FP64 network oracle (Sec. 3.3 post-processor, reduced to the
encoder-decoder this build trains): each layer against torch's CPU float64
library routines (an independent implementation), the whole forward pass
against a torch re-composition, gradients against central finite
differences, and Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import net as onet



def T(a):
    return torch.from_numpy(np.ascontiguousarray(a))


@pytest.mark.parametrize("k,ci,co", [(3, 5, 7), (3, 8, 32), (1, 32, 3)])
def test_conv_matches_torch(k, ci, co):
    rng = np.random.default_rng(k * 100 + ci)
    x = rng.standard_normal((2, ci, 9, 12))
    Wt = rng.standard_normal((co, ci, k, k))
    b = rng.standard_normal(co)
    y, _ = onet.conv(x, Wt, b)
    ref = F.conv2d(T(x), T(Wt), T(b), padding=k // 2).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_pool_and_upsample_match_torch():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 8, 10))
    np.testing.assert_allclose(onet.avgpool2(x), F.avg_pool2d(T(x), 2).numpy(), rtol=1e-14, atol=1e-14)
    up = F.interpolate(T(x), scale_factor=2, mode="bilinear", align_corners=False).numpy()
    np.testing.assert_allclose(onet.upsample2(x), up, rtol=1e-13, atol=1e-13)
    # constants stay constant, ramps stay linear in the interior
    c = np.full((1, 1, 4, 4), 2.5)
    np.testing.assert_allclose(onet.upsample2(c), 2.5, rtol=0, atol=1e-15)
    np.testing.assert_allclose(onet.avgpool2(c), 2.5, rtol=0, atol=0)


def torch_forward(P, x):
    def cv(n, t, act=True):
        Wt, b = P[n]
        z = F.conv2d(t, T(Wt), T(b), padding=Wt.shape[2] // 2)
        return F.relu(z) if act else z
    up = lambda t: F.interpolate(t, scale_factor=2, mode="bilinear", align_corners=False)
    s1 = cv("e1b", cv("e1a", T(x)))
    s2 = cv("e2b", cv("e2a", F.avg_pool2d(s1, 2)))
    s3 = cv("e3b", cv("e3a", F.avg_pool2d(s2, 2)))
    s4 = cv("e4b", cv("e4a", F.avg_pool2d(s3, 2)))
    d3 = cv("d3b", cv("d3a", torch.cat([up(s4), s3], 1)))
    d2 = cv("d2b", cv("d2a", torch.cat([up(d3), s2], 1)))
    d1 = cv("d1b", cv("d1a", torch.cat([up(d2), s1], 1)))
    return cv("head", d1, act=False)


def test_forward_matches_torch_full_width():
    rng = np.random.default_rng(2)
    P = onet.init_params(rng)
    for name, (Wt, b) in P.items():
        P[name] = (Wt, rng.standard_normal(b.shape) * 0.1)
    x = rng.random((1, 8, 16, 24))
    y, _ = onet.forward(P, x)
    np.testing.assert_allclose(y, torch_forward(P, x).detach().numpy(), rtol=1e-10, atol=1e-10)


def test_backward_matches_torch_autograd():
    rng = np.random.default_rng(3)
    table = onet.layer_table((4, 8, 8, 16))
    P = onet.init_params(rng, table)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((2, 8, 16, 16))
    t = rng.random((2, 3, 16, 16))
    y, cache = onet.forward(P, x)
    L, dy = onet.loss(y, t, lam_tv=1e-2)
    G = onet.backward(P, cache, dy)
    # torch autograd on the same composition
    Pt = {k: (T(w).requires_grad_(), T(b).requires_grad_()) for k, (w, b) in P.items()}

    def cv(n, tt, act=True):
        Wt, b = Pt[n]
        z = F.conv2d(tt, Wt, b, padding=Wt.shape[2] // 2)
        return F.relu(z) if act else z
    up = lambda tt: F.interpolate(tt, scale_factor=2, mode="bilinear", align_corners=False)
    s1 = cv("e1b", cv("e1a", T(x)))
    s2 = cv("e2b", cv("e2a", F.avg_pool2d(s1, 2)))
    s3 = cv("e3b", cv("e3a", F.avg_pool2d(s2, 2)))
    s4 = cv("e4b", cv("e4a", F.avg_pool2d(s3, 2)))
    d3 = cv("d3b", cv("d3a", torch.cat([up(s4), s3], 1)))
    d2 = cv("d2b", cv("d2a", torch.cat([up(d3), s2], 1)))
    d1 = cv("d1b", cv("d1a", torch.cat([up(d2), s1], 1)))
    yt = cv("head", d1, act=False)
    tt = T(t)
    Lt = ((yt - tt) ** 2).mean() + 1e-2 * ((yt[..., 1:] - yt[..., :-1]).abs().mean()
                                            + (yt[..., 1:, :] - yt[..., :-1, :]).abs().mean())
    Lt.backward()
    assert abs(float(Lt) - L) < 1e-12
    for k, (w, b) in Pt.items():
        np.testing.assert_allclose(G[k][0], w.grad.numpy(), rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(G[k][1], b.grad.numpy(), rtol=1e-9, atol=1e-12)


def test_gradients_by_finite_differences():
    rng = np.random.default_rng(4)
    table = onet.layer_table((4, 8, 8, 16), in_ch=8, out_ch=3)
    P = onet.init_params(rng, table)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((1, 8, 16, 16))
    t = rng.random((1, 3, 16, 16))

    def Lof(PP):
        y, _ = onet.forward(PP, x)
        return onet.loss(y, t, lam_tv=0.0)[0]
    y, cache = onet.forward(P, x)
    _, dy = onet.loss(y, t, lam_tv=0.0)
    G = onet.backward(P, cache, dy)
    h = 1e-6
    for name in ("e1a", "e3b", "e4a", "d3a", "d1b", "head"):
        Wt, b = P[name]
        for _ in range(4):
            idx = tuple(rng.integers(0, s) for s in Wt.shape)
            Wp, Wm = Wt.copy(), Wt.copy()
            Wp[idx] += h
            Wm[idx] -= h
            num = (Lof({**P, name: (Wp, b)}) - Lof({**P, name: (Wm, b)})) / (2 * h)
            assert abs(num - G[name][0][idx]) <= 1e-6 * max(1e-3, abs(num)), (name, idx, num, G[name][0][idx])
        j = int(rng.integers(0, b.shape[0]))
        bp, bm = b.copy(), b.copy()
        bp[j] += h
        bm[j] -= h
        num = (Lof({**P, name: (Wt, bp)}) - Lof({**P, name: (Wt, bm)})) / (2 * h)
        assert abs(num - G[name][1][j]) <= 1e-6 * max(1e-3, abs(num))


def test_adam_matches_torch():
    rng = np.random.default_rng(5)
    P = {"a": (rng.standard_normal((3, 2, 1, 1)), rng.standard_normal(3))}
    p_w, p_b = T(P["a"][0].copy()).requires_grad_(), T(P["a"][1].copy()).requires_grad_()
    opt = torch.optim.Adam([p_w, p_b], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    state = {}
    for _ in range(3):
        gw, gb = rng.standard_normal((3, 2, 1, 1)), rng.standard_normal(3)
        P = onet.adam(P, {"a": (gw, gb)}, state)
        opt.zero_grad()
        p_w.grad, p_b.grad = T(gw), T(gb)
        opt.step()
    np.testing.assert_allclose(P["a"][0], p_w.detach().numpy(), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(P["a"][1], p_b.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_psnr():
    a = np.zeros((3, 4, 4))
    assert onet.psnr(a, a) == float("inf")
    assert onet.psnr(a, a + 0.1) == pytest.approx(20.0)


def test_features_hand_computed_fixture():
    """features(): a 2 x 2 image computed by hand (tests/golden/features_2x2.txt):
    depth d > 0 becomes 1/d, an empty pixel (d = 0) gives 0, the other seven
    planes are unchanged."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "features_2x2.txt")
    rows = {"in": [], "out": []}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        kind, _name, *vals = line.split()
        rows[kind].append([float(v) for v in vals])
    x = np.array(rows["in"]).reshape(1, 8, 2, 2)
    want = np.array(rows["out"]).reshape(1, 8, 2, 2)
    np.testing.assert_array_equal(onet.features(x), want)
    # the input array itself is left untouched
    assert x[0, 3, 0, 0] == 2.0


def test_crop_forward_equals_full_forward():
    """The crop procedure the 1920 x 1080 parity test relies on: a tile's
    outputs computed on a crop with the margin equal the full-image outputs
    (narrow layers: the reach of an output depends on the depth only), at
    the border and inside; a margin far below the reach does not."""
    import netcheck
    rng = np.random.default_rng(5)
    table = onet.layer_table(widths=(4, 4, 4, 8), in_ch=8, out_ch=3)
    P = onet.init_params(rng, table)
    P = {k: (w, rng.standard_normal(b.shape) * 0.1) for k, (w, b) in P.items()}
    x = rng.random((1, 8, 240, 304))
    full, _ = onet.forward(P, x)
    for (y0, y1, x0, x1) in [(0, 32, 0, 48), (104, 136, 128, 176), (208, 240, 264, 304)]:
        tile = netcheck.crop_forward(P, x, y0, y1, x0, x1)
        np.testing.assert_allclose(tile, full[:, :, y0:y1, x0:x1], rtol=0, atol=1e-12)
    short = netcheck.crop_forward(P, x, 104, 136, 128, 176, margin=16)
    assert np.abs(short - full[:, :, 104:136, 128:176]).max() > 1e-6
