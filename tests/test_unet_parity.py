"""The paper's gated U-Net on the GPU against the FP64 oracle (oracle/unet.py).

Forward: bf16 operands and activations, fp32 accumulation, within 2e-2
max-abs of the FP64 forward on the fp32 parameters (the bf16 bound of the
network contract), on frames on and off the 16-pixel grid.  Gradients: every layer's weight and bias gradient within
a normwise relative bound of the FP64 backward fed the same bf16-rounded
parameters and input; the GPU stores every activation and gradient tensor in
bf16 (2^-9 relative each), and the gating's products chain about a dozen such
roundings along the longest path, so the bound is 3e-2 normwise (measured
errors are printed).  Training: Adam steps on one batch lower the loss."""
import numpy as np
import pytest

from oracle import net as onet
from oracle import unet as ounet
from paper_2407_19097_amd import narvis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = (32, 32, 64, 64, 64)


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def random_unet(seed, widths, out_scale=0.3):
    rng = np.random.default_rng(seed)
    P = ounet.init_params(rng, widths)
    P = {k: (w, rng.standard_normal(b.shape) * 0.05) for k, (w, b) in P.items()}
    Wh, bh = P["head"]
    P["head"] = (Wh * out_scale, bh + 0.5)
    return P


def random_planes(rng, B, H, W):
    x = rng.random((B, 8, H, W)).astype(np.float32)
    x[:, 3] = (0.5 + x[:, 3] * 4.0).astype(np.float32)  # depth in [0.5, 4.5]
    x[:, 3][rng.random((B, H, W)) < 0.2] = 0.0          # empty pixels
    return x


def bf16(a):
    return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


@pytest.mark.parametrize("widths,B,H,W", [(SMALL, 2, 32, 48), (SMALL, 1, 64, 80), (ounet.WIDTHS, 1, 32, 32),
                                           (SMALL, 1, 36, 50), (SMALL, 2, 17, 40)])
def test_unet_forward_matches_oracle(widths, B, H, W):
    announce(f"gated U-Net forward, widths {widths}, B={B} {H}x{W}")
    P = random_unet(B * 31 + H, widths)
    planes = random_planes(np.random.default_rng(W), B, H, W)
    u = narvis.UNet(ounet.to_blob(P, widths).astype(np.float32), widths)
    ws = torch.empty(narvis.narvis_unet_workspace_size(u, B, W, H), dtype=torch.uint8, device="cuda")
    img = torch.empty((B, 3, H, W), dtype=torch.float32, device="cuda")
    narvis.narvis_unet_forward(u, torch.from_numpy(planes).cuda(), B, W, H, img, ws)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    want = ounet.infer(P, onet.features(planes))  # frames off the 16 grid: zero-padded, cropped
    err = float(np.abs(got - want).max())
    print(f"  max |gpu - fp64| = {err:.4g}, output range [{want.min():.2f}, {want.max():.2f}]", flush=True)
    assert np.isfinite(got).all()
    assert err <= 2e-2
    u.close()


@pytest.mark.parametrize("B,H,W", [(2, 32, 48), (1, 48, 32)])
def test_unet_gradients_match_oracle(B, H, W):
    announce(f"gated U-Net gradients per layer, widths {SMALL}, B={B} {H}x{W}")
    P = random_unet(7 + H, SMALL)
    rng = np.random.default_rng(H + W)
    planes = random_planes(rng, B, H, W)
    target = rng.random((B, 3, H, W)).astype(np.float32)
    blob = ounet.to_blob(P, SMALL).astype(np.float32)
    u = narvis.UNet(blob, SMALL)
    ws = torch.empty(narvis.narvis_unet_workspace_size(u, B, W, H, train=True), dtype=torch.uint8, device="cuda")
    grad = torch.empty(blob.size, dtype=torch.float32, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    narvis.narvis_unet_gradients(u, torch.from_numpy(planes).cuda(), torch.from_numpy(target).cuda(), B, W, H, 1e-3,
                                 grad, lossv, ws)
    torch.cuda.synchronize()
    g = ounet.from_blob(grad.cpu().numpy().astype(np.float64), SMALL)
    # the oracle on the bf16-rounded parameters and input the GPU used
    Pb = ounet.from_blob(bf16(blob), SMALL)
    x = bf16(onet.features(planes))
    y, cache = ounet.forward(Pb, x)
    L, gy = onet.loss(y, target.astype(np.float64), lam_tv=1e-3)
    G = ounet.backward(Pb, cache, gy)
    print(f"  loss gpu {float(lossv.item()):.6f} oracle {L:.6f}", flush=True)
    assert abs(float(lossv.item()) - L) <= 1e-2 * L
    worst = 0.0
    for name, *_ in ounet.layers(SMALL):
        for k in (0, 1):
            a, b = g[name][k], G[name][k]
            rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
            worst = max(worst, rel)
            assert rel <= 3e-2, (name, k, rel)
    print(f"  worst normwise relative gradient error {worst:.3g}", flush=True)
    u.close()


def test_unet_training_lowers_the_loss():
    announce("gated U-Net: 40 Adam steps on one batch")
    B, H, W = 4, 32, 32
    P = random_unet(3, SMALL)
    rng = np.random.default_rng(5)
    planes = torch.from_numpy(random_planes(rng, B, H, W)).cuda()
    target = planes[:, :3].clone()
    u = narvis.UNet(ounet.to_blob(P, SMALL).astype(np.float32), SMALL)
    ws = torch.empty(narvis.narvis_unet_workspace_size(u, B, W, H, train=True), dtype=torch.uint8, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for _ in range(40):
        narvis.narvis_unet_train_step(u, planes, target, B, W, H, 1e-3, 1e-3, lossv, ws)
        losses.append(float(lossv.item()))
    print(f"  loss {losses[0]:.5f} -> {losses[-1]:.5f}", flush=True)
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.5 * losses[0]
    u.close()


@pytest.mark.timeout(600)
def test_unet_trained_forward_1080p(c4_net):
    """The gated U-Net trained by the shared fixture, on a held-out view at
    1920 x 1080: the GPU runs the whole frame; the FP64 oracle runs the three
    256 x 256 crops (origins on a 64-pixel grid, so on the 16-pixel pooling
    grid) whose centres hold the most covered pixels, and the centre 64 x 64
    of each is compared.  A changed input pixel moves outputs up to 47 pixels
    away (measured on the oracle for a pixel at the start of a 16-pixel
    block; at most 15 more elsewhere in the block), less than the 96-pixel
    margin, so those outputs see no crop border."""
    from paper_2407_19097_amd import train
    announce("trained gated U-Net, held-out view at 1920x1080 vs the FP64 oracle on the three most covered "
             "256x256 crops")
    sc, u = c4_net["scene"], c4_net["unet"]
    W, H = 1920, 1080
    r = train.Renderer(sc, W, H)
    feat = torch.empty((8, H * W), dtype=torch.float32, device="cuda")
    r.gbuffer(c4_net["heldout"][0], feat)
    img = torch.empty((1, 3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(narvis.narvis_unet_workspace_size(u, 1, W, H), dtype=torch.uint8, device="cuda")
    narvis.narvis_unet_forward(u, feat.view(1, 8, H * W), 1, W, H, img, ws)
    torch.cuda.synchronize()
    planes = feat.view(1, 8, H, W).cpu().numpy()
    got = img.cpu().numpy().astype(np.float64)
    P = ounet.from_blob(u.read().astype(np.float64), ounet.WIDTHS)
    # the three crops (origins on a 64-pixel grid) whose compared centres hold
    # the most covered pixels
    cov = planes[0, 3] > 0
    cands = [(int(cov[y + 96:y + 160, x + 96:x + 160].sum()), y, x)
             for y in range(0, H - 256 + 1, 64) for x in range(0, W - 256 + 1, 64)]
    crops = [(y, x) for _, y, x in sorted(cands, reverse=True)[:3]]
    print(f"  crops {crops}, covered centre pixels {[c for c, *_ in sorted(cands, reverse=True)[:3]]}", flush=True)
    worst = 0.0
    for y0, x0 in crops:
        x = onet.features(planes[:, :, y0:y0 + 256, x0:x0 + 256])
        want = ounet.forward(P, x)[0][:, :, 96:160, 96:160]
        err = float(np.abs(got[:, :, y0 + 96:y0 + 160, x0 + 96:x0 + 160] - want).max())
        print(f"  crop ({y0}, {x0}): max |gpu - fp64| = {err:.4g}, output range [{want.min():.2f}, {want.max():.2f}]",
              flush=True)
        worst = max(worst, err)
    assert worst <= 2e-2
