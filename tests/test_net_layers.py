"""Training path of the network, layer by layer, element by element, against
the FP64 oracle.

After one narvis_train_gradients call every tensor the GPU stored in its
workspace (each layer's bf16 input and output, the pooled and upsampled
tensors, every gradient) is read back.  Each step is then recomputed in FP64
by the oracle from the GPU's own stored inputs and the bf16-rounded
parameters the GPU used, so the only differences left are the GPU's fp32
accumulation order and, for stored bf16 tensors, the final rounding:

  |gpu - exact| <= 2^-8 |exact|                      (bf16 round to nearest)
                 + 2 (K + 2) 2^-24 sum_k |t_k| (1 + 2^-8)  (fp32 accumulation
                   of the K exact bf16 x bf16 products t_k, any order; the
                   factor 2 also covers a truncating accumulator)

with K the number of terms of that element (9 Cin + 1 for a 3x3 forward
output, 9 Cout for an input gradient, the pixel count for a weight or bias
gradient).  Weight and bias gradients are fp32 outputs (no bf16 term) and
must also agree within 1e-3 normwise (the network-gradient bound of the
oracle's contract); in practice they agree to about 1e-6.

The wiring of each step (which stored tensor is a layer's input, output and
upstream gradient) follows the network's definition, so a kernel that reads
the wrong tensor fails here as well."""
import numpy as np
import pytest

from oracle import net as onet
from paper_2407_19097_amd import narvis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
U16 = 2.0 ** -8

# (layer, input tensors, output tensor, gradient of the output, gradient of the input)
CONV_STEPS = [
    ("e1a", ["feat"], "e1a", "g_e1a", None),
    ("e1b", ["e1a"], "sk1", "g_e1b", "g_e1a"),
    ("e2a", ["pool1"], "e2a", "g_e2a", "g_pool1"),
    ("e2b", ["e2a"], "sk2", "g_e2b", "g_e2a"),
    ("e3a", ["pool2"], "e3a", "g_e3a", "g_pool2"),
    ("e3b", ["e3a"], "sk3", "g_e3b", "g_e3a"),
    ("e4a", ["pool3"], "e4a", "g_e4a", "g_pool3"),
    ("e4b", ["e4a"], "e4b", "g_e4b", "g_e4a"),
    ("d3a", ["up3", "sk3"], "d3a", "g_d3a", "g_cat3"),
    ("d3b", ["d3a"], "d3b", "g_d3b", "g_d3a"),
    ("d2a", ["up2", "sk2"], "d2a", "g_d2a", "g_cat2"),
    ("d2b", ["d2a"], "d2b", "g_d2b", "g_d2a"),
    ("d1a", ["up1", "sk1"], "d1a", "g_d1a", "g_cat1"),
    ("d1b", ["d1a"], "d1b", "g_d1b", "g_d1a"),
    ("head", ["d1b"], "out", "gy", "g_d1b"),
]
POOLS = [("pool1", "sk1"), ("pool2", "sk2"), ("pool3", "sk3")]
UPS = [("up3", "e4b"), ("up2", "d3b"), ("up1", "d2b")]
# gradient of a lower-resolution tensor from the upsampled part of a concat gradient
UP_BWD = [("g_e4b", "g_cat3", 256), ("g_d3b", "g_cat2", 128), ("g_d2b", "g_cat1", 64)]
# gradient of a skip tensor: pooled path + the skip part of the concat gradient
POOL_BWD = [("g_e3b", "g_pool3", "g_cat3", 256), ("g_e2b", "g_pool2", "g_cat2", 128),
            ("g_e1b", "g_pool1", "g_cat1", 64)]


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def bf16_round(a):
    t = torch.from_numpy(np.asarray(a, np.float32).copy()).to(torch.bfloat16)
    return t.to(torch.float64).numpy()


def random_net(seed, out_scale=0.3):
    rng = np.random.default_rng(seed)
    P = onet.init_params(rng)
    P = {k: (w, rng.standard_normal(b.shape) * 0.05) for k, (w, b) in P.items()}
    Wh, bh = P["head"]
    P["head"] = (Wh * out_scale, bh + 0.5)
    return P


def random_planes(rng, B, H, W):
    planes = rng.random((B, 8, H, W)).astype(np.float32)
    planes[:, 3] = (0.5 + 3 * rng.random((B, H, W))).astype(np.float32)
    planes[:, 3][rng.random((B, H, W)) < 0.2] = 0.0
    planes[:, 4:6] = (rng.standard_normal((B, 2, H, W)) * 0.5).astype(np.float32)
    planes[:, 6] = (rng.random((B, H, W)) * 2 - 1).astype(np.float32)
    return planes


class Stored:
    """Tensors of the training workspace as float64 NCHW arrays."""

    def __init__(self, ws, B, W, H):
        self.ws, self.B, self.W, self.H = ws, B, W, H
        self.host = ws.cpu()

    def __getitem__(self, name):
        off, c, h, w, dt = narvis.narvis_train_tensor(self.B, self.W, self.H, name)
        if dt == 1:
            n = self.B * c * h * w * 4
            return self.host[off:off + n].view(torch.float32).view(self.B, c, h, w).double().numpy()
        n = self.B * h * w * c * 2
        t = self.host[off:off + n].view(torch.bfloat16).view(self.B, h, w, c)
        return t.permute(0, 3, 1, 2).double().numpy()


def check(what, got, exact, absterms, K, bf16_out):
    bound = 2 * (K + 2) * U32 * absterms * (1 + U16)
    if bf16_out:
        bound = bound + U16 * np.abs(exact)
    err = np.abs(got - exact)
    bad = err > bound
    assert not bad.any(), (f"{what}: {int(bad.sum())} of {bad.size} elements out of bound, worst "
                           f"{float((err - bound).max()):.3g} over")
    rel = float(np.linalg.norm(got - exact) / max(np.linalg.norm(exact), 1e-30))
    return rel


def run_case(B, H, W, seed):
    P = random_net(seed)
    rng = np.random.default_rng(seed + 1)
    planes = random_planes(rng, B, H, W)
    target = rng.random((B, 3, H, W)).astype(np.float32)
    blob32 = onet.to_blob(P).astype(np.float32)
    w = narvis.NetWeights(blob32)
    ws = torch.zeros(narvis.narvis_train_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    grad = torch.empty(blob32.size, dtype=torch.float32, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    lam = 1e-3
    narvis.narvis_train_gradients(w, torch.from_numpy(planes).cuda(), torch.from_numpy(target).cuda(), B, W, H,
                                  lam, grad, lossv, ws)
    torch.cuda.synchronize()
    S = Stored(ws, B, W, H)
    G_gpu = onet.from_blob(grad.cpu().numpy().astype(np.float64))
    # the parameters as the GPU used them: bf16 weights, fp32 biases
    Pq = onet.from_blob(blob32.astype(np.float64))
    Wq = {k: (bf16_round(wt), b) for k, (wt, b) in Pq.items()}
    w.close()
    worst = {"fwd": 0.0, "dx": 0.0, "dW": 0.0, "db": 0.0}

    # network input: depth inverted, rounded to bf16
    feat = S["feat"]
    np.testing.assert_array_equal(feat, bf16_round(onet.features(planes)))

    # loss and its gradient from the GPU's own fp32 output
    out = S["out"]
    L, gy = onet.loss(out, target.astype(np.float64), lam_tv=lam)
    assert abs(float(lossv.item()) - L) <= 1e-4 * L, (float(lossv.item()), L)
    gy_gpu = S["gy"]
    assert (gy_gpu[:, 3:] == 0).all()
    n_all = out.size
    terms = 2.0 * np.abs(out - target) / n_all + 4 * lam / min(B * 3 * H * (W - 1), B * 3 * (H - 1) * W)
    check("loss gradient", gy_gpu[:, :3], gy, terms, 5, True)

    for name, src in POOLS:
        x = S[src]
        check(f"pool {name}", S[name], onet.avgpool2(x), onet.avgpool2(np.abs(x)), 4, True)
    for name, src in UPS:
        x = S[src]
        check(f"upsample {name}", S[name], onet.upsample2(x), onet.upsample2(np.abs(x)), 4, True)
    for name, src, c in UP_BWD:
        g = S[src][:, :c]
        check(f"upsample backward {name}", S[name], onet.upsample2_backward(g),
              onet.upsample2_backward(np.abs(g)), 16, True)
    for name, gp, cat, c in POOL_BWD:
        a, b = S[gp], S[cat][:, c:]
        check(f"pool backward + skip {name}", S[name], onet.avgpool2_backward(a) + b,
              onet.avgpool2_backward(np.abs(a)) + np.abs(b), 2, True)

    for layer, xs, own_name, dy_name, dx_name in CONV_STEPS:
        x = np.concatenate([S[n] for n in xs], axis=1)
        Wt, b = Wq[layer]
        relu = layer != "head"
        k = Wt.shape[2]
        cin, cout = Wt.shape[1], Wt.shape[0]
        # forward: the stored output from the stored input
        z, cols = onet.conv(x, Wt, b)
        za, _ = onet.conv(np.abs(x), np.abs(Wt), np.abs(b))
        own = S[own_name]
        want = onet.relu(z) if relu else z
        worst["fwd"] = max(worst["fwd"], check(f"{layer} forward", own, want, za, k * k * cin + 1, relu))
        # backward: upstream gradient masked by the stored output
        dy = S[dy_name][:, :cout]
        g = dy * (own > 0) if relu else dy
        dx, dW, db = onet.conv_backward(g, cols, Wt, x.shape)
        _, colsa = onet.conv(np.abs(x), np.abs(Wt), np.abs(b))
        dxa, dWa, dba = onet.conv_backward(np.abs(g), colsa, np.abs(Wt), x.shape)
        npx = B * x.shape[2] * x.shape[3]
        rW = check(f"{layer} weight gradient", G_gpu[layer][0], dW, dWa, npx, False)
        rb = check(f"{layer} bias gradient", G_gpu[layer][1], db, dba, npx, False)
        assert rW <= 1e-3 and rb <= 1e-3, (layer, rW, rb)
        worst["dW"] = max(worst["dW"], rW)
        worst["db"] = max(worst["db"], rb)
        if dx_name is not None:
            worst["dx"] = max(worst["dx"], check(f"{layer} input gradient", S[dx_name], dx, dxa,
                                                 k * k * cout, True))
    print("  worst normwise relative error: " + ", ".join(f"{k} {v:.2e}" for k, v in worst.items()), flush=True)
    return worst


@pytest.mark.parametrize("B,H,W", [(2, 32, 48), (1, 40, 24)])
def test_every_layer_forward_and_backward_against_oracle(B, H, W):
    announce(f"network training path layer by layer B={B} {H}x{W}")
    run_case(B, H, W, seed=7 + H)
