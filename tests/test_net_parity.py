"""GPU network (bf16 implicit-GEMM convolutions on MFMA, fp32 accumulation)
against the FP64 oracle.

Forward: within 2e-2 max-abs of the FP64 forward on the fp32 parameters for
outputs scaled to about [0, 1].  Adam: exact update rule against the oracle
given the GPU's own gradients (fp32 vs fp64, 1e-5 relative).  Training:
the loss curve of 60 steps on one batch against the FP64 oracle's.  The
gradients are checked layer by layer in test_net_layers.py."""
import numpy as np
import pytest

from oracle import net as onet
from paper_2407_19097_amd import narvis

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"\n[case] {msg}", flush=True)


def bf16_round(a):
    """Round float64/float32 values to bfloat16 (nearest even), back to float64."""
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
    planes[:, 3] = (0.5 + 3 * rng.random((B, H, W))).astype(np.float32)  # depth
    planes[:, 3][rng.random((B, H, W)) < 0.2] = 0.0                        # empty pixels
    planes[:, 4:6] = (rng.standard_normal((B, 2, H, W)) * 0.5).astype(np.float32)
    planes[:, 6] = (rng.random((B, H, W)) * 2 - 1).astype(np.float32)
    return planes


def gpu_forward(P, planes):
    B, _, H, W = planes.shape
    w = narvis.NetWeights(onet.to_blob(P).astype(np.float32))
    feat = torch.from_numpy(planes).cuda()
    img = torch.empty((B, 3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(narvis.narvis_postprocess_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    narvis.narvis_postprocess(w, feat, B, W, H, img, ws)
    torch.cuda.synchronize()
    out = img.cpu().numpy().astype(np.float64)
    w.close()
    return out


@pytest.mark.parametrize("B,H,W", [(1, 8, 8), (2, 32, 48), (1, 64, 64), (1, 136, 240)])
def test_forward_matches_oracle(B, H, W):
    announce(f"network forward B={B} {H}x{W}")
    P = random_net(B * 1000 + H)
    rng = np.random.default_rng(H + W)
    planes = random_planes(rng, B, H, W)
    got = gpu_forward(P, planes)
    want, _ = onet.forward(P, onet.features(planes))
    err = np.abs(got - want).max()
    print(f"  max |gpu - fp64| = {err:.3g}, output range [{want.min():.2f}, {want.max():.2f}]", flush=True)
    assert np.isfinite(got).all()
    assert err <= 2e-2


def test_adam_step_and_determinism():
    announce("train step: Adam update against the oracle, bit-reproducible")
    B, H, W = 2, 16, 16
    P = random_net(11)
    rng = np.random.default_rng(12)
    planes = torch.from_numpy(random_planes(rng, B, H, W)).cuda()
    target = torch.from_numpy(rng.random((B, 3, H, W)).astype(np.float32)).cuda()
    blob32 = onet.to_blob(P).astype(np.float32)
    ws = torch.empty(narvis.narvis_train_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    grad = torch.empty(blob32.size, dtype=torch.float32, device="cuda")
    w = narvis.NetWeights(blob32)
    narvis.narvis_train_gradients(w, planes, target, B, W, H, 1e-3, grad, lossv, ws)
    narvis.narvis_train_step(w, planes, target, B, W, H, 1e-3, 1e-3, lossv, ws)
    torch.cuda.synchronize()
    after = w.read()
    g = onet.from_blob(grad.cpu().numpy())
    want = onet.to_blob(onet.adam(onet.from_blob(blob32), g, {}, lr=1e-3))
    np.testing.assert_allclose(after, want, rtol=1e-5, atol=1e-7)
    w2 = narvis.NetWeights(blob32)
    narvis.narvis_train_step(w2, planes, target, B, W, H, 1e-3, 1e-3, lossv, ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(w2.read().view(np.uint32), after.view(np.uint32))
    w.close()
    w2.close()


def test_training_follows_oracle_loss_curve():
    """60 Adam steps on one batch: the loss before steps 1, 20, 40 and 60
    stays within 10 % of the FP64 oracle trained the same way (the GPU
    trains with bf16 operands, so the curves drift apart slowly), and halves
    (the oracle reaches 0.35 x the initial loss by step 60)."""
    announce("60 Adam steps on one batch follow the oracle's loss curve")
    import json
    import os
    B, H, W = 4, 32, 32
    P = random_net(13)
    rng = np.random.default_rng(14)
    planes = torch.from_numpy(random_planes(rng, B, H, W)).cuda()
    target = planes[:, :3].clone()
    w = narvis.NetWeights(onet.to_blob(P).astype(np.float32))
    ws = torch.empty(narvis.narvis_train_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    losses = []
    for _ in range(60):
        narvis.narvis_train_step(w, planes, target, B, W, H, 1e-3, 0.0, lossv, ws)
        losses.append(float(lossv.item()))
    w.close()
    golden = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "train_curve.json")))
    print(f"  loss {losses[0]:.4f} -> {losses[-1]:.4f}", flush=True)
    assert all(np.isfinite(losses))
    for k, want in golden["loss_before_step"].items():
        got = losses[int(k) - 1]
        print(f"  before step {k}: gpu {got:.5f} oracle {want:.5f}", flush=True)
        assert abs(got - want) <= 0.1 * want, (k, got, want)
    assert losses[-1] < 0.5 * losses[0]


@pytest.mark.parametrize("B,H,W", [(1, 32, 32), (2, 64, 96)])
def test_fp8_forward_matches_oracle(B, H, W):
    """FP8 (e4m3, per-output-channel weight scales, static per-layer
    activation scales calibrated on another batch drawn from the same
    distribution; the layers the calibration chose in FP8, the rest in bf16)
    within 6e-2 max-abs of the FP64 forward."""
    announce(f"FP8 network forward B={B} {H}x{W}")
    P = random_net(B * 77 + H)
    rng = np.random.default_rng(W + 5)
    planes = random_planes(rng, B, H, W)
    w = narvis.NetWeights(onet.to_blob(P).astype(np.float32))
    feat = torch.from_numpy(planes).cuda()
    ws = torch.empty(narvis.narvis_train_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    img = torch.empty((B, 3, H, W), dtype=torch.float32, device="cuda")
    with pytest.raises(narvis.NarvisError):
        narvis.narvis_postprocess(w, feat, B, W, H, img, ws, precision=narvis.PRECISION_FP8)
    cal = torch.from_numpy(random_planes(np.random.default_rng(W + 1005), B, H, W)).cuda()
    narvis.narvis_weights_calibrate_fp8(w, cal, B, W, H, ws)
    mask = narvis.narvis_weights_fp8_layers(w)
    narvis.narvis_postprocess(w, feat, B, W, H, img, ws, precision=narvis.PRECISION_FP8)
    torch.cuda.synchronize()
    got = img.cpu().numpy().astype(np.float64)
    want, _ = onet.forward(P, onet.features(planes))
    err = np.abs(got - want).max()
    print(f"  FP8 layers {fp8_names(mask)}; max |gpu - fp64| = {err:.3g}", flush=True)
    assert mask != 0
    assert np.isfinite(got).all()
    assert err <= 6e-2
    w.close()


def oracle_planes(sc, cam, W, H):
    """G-buffer planes [8][H][W] (r, g, b, depth, v'x, v'y, theta, |v'|) of one
    view rendered by the CPU raster oracle from the scene's seeded arrays."""
    from oracle import camera as ocam
    from oracle import raster as orast
    from paper_2407_19097_amd import scenes
    x, y, z = (t.cpu().numpy() for t in (sc.x, sc.y, sc.z))
    attrs = [a.cpu().numpy() for a in sc.attrs]
    M, near, far = ocam.clip_matrix(cam, W, H)
    keys = orast.render(x, y, z, M, near, far, W, H)
    o = orast.resolve(keys, W, H, x, y, z, M, attrs, want_attrs=False, lut=scenes.colour_lut(),
                      lut_attr=sc.lut_attr, lut_min=sc.lut_min,
                      lut_inv_range=float(np.float32(1.0 / (sc.lut_max - sc.lut_min))), vel_attr=sc.vel_attr)
    return np.concatenate([o["rgb"], o["depth"][None], o["vel2d"]]).reshape(8, H, W)


def gpu_trained_forward(w, planes, precision):
    B, _, H, W = planes.shape
    img = torch.empty((B, 3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(narvis.narvis_postprocess_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    narvis.narvis_postprocess(w, torch.from_numpy(planes).cuda(), B, W, H, img, ws, precision=precision)
    torch.cuda.synchronize()
    return img.cpu().numpy().astype(np.float64)


LAYER_NAMES = [n for n, *_ in onet.LAYERS]


def fp8_names(mask):
    return [n for i, n in enumerate(LAYER_NAMES) if (mask >> i) & 1]


def calibrate_on_training_views(c4):
    """FP8 calibration on 16 training views (never the tested ones); returns
    the chosen layer mask, which must put at least one layer in FP8."""
    cal = c4["cal"]
    B, _, H, W = cal.shape
    ws = torch.empty(narvis.narvis_train_workspace_size(B, W, H), dtype=torch.uint8, device="cuda")
    narvis.narvis_weights_calibrate_fp8(c4["weights"], cal, B, W, H, ws)
    torch.cuda.synchronize()
    mask = narvis.narvis_weights_fp8_layers(c4["weights"])
    print(f"  FP8 layers chosen on the training views: {fp8_names(mask)}", flush=True)
    assert mask != 0
    return mask


@pytest.mark.timeout(900)
def test_trained_forward_on_heldout_views_512(c4_net):
    """Trained weights on two held-out views at 512 x 512 (G-buffers from the
    CPU raster oracle): BF16 within 2e-2 and FP8 (activation scales from 16
    training views) within 6e-2 max-abs of the FP64 forward on the fp32
    master parameters, over every output."""
    announce("trained network, 2 held-out vector-field views 512x512, BF16 and FP8")
    w = c4_net["weights"]
    P = onet.from_blob(w.read().astype(np.float64))
    planes = np.stack([oracle_planes(c4_net["scene"], cam, 512, 512) for cam in c4_net["heldout"][:2]])
    want, _ = onet.forward(P, onet.features(planes))
    calibrate_on_training_views(c4_net)
    for prec, bound in ((narvis.PRECISION_BF16, 2e-2), (narvis.PRECISION_FP8, 6e-2)):
        got = gpu_trained_forward(w, planes, prec)
        err = float(np.abs(got - want).max())
        print(f"  {'BF16' if prec == 0 else 'FP8'}: max |gpu - fp64| = {err:.4f} (bound {bound}, margin "
              f"{bound - err:.4f}); output range [{want.min():.2f}, {want.max():.2f}]", flush=True)
        assert np.isfinite(got).all()
        assert err <= bound


@pytest.mark.timeout(900)
def test_trained_forward_at_1080p_on_crops(c4_net):
    """Trained weights on a held-out view at 1920 x 1080: the GPU runs the
    whole frame (BF16, then FP8 calibrated on training views); the FP64
    oracle computes three 64 x 64 output tiles (top-left corner, centre,
    bottom-right corner) on crops that carry the full receptive field."""
    import netcheck
    announce("trained network, held-out vector-field view 1920x1080, BF16 and FP8 on three tiles")
    W, H = 1920, 1080
    w = c4_net["weights"]
    P = onet.from_blob(w.read().astype(np.float64))
    planes = oracle_planes(c4_net["scene"], c4_net["heldout"][2], W, H)[None]
    x = onet.features(planes)
    tiles = [(0, 64, 0, 64), (512, 576, 928, 992), (H - 64, H, W - 64, W)]
    wants = [netcheck.crop_forward(P, x, *t) for t in tiles]
    calibrate_on_training_views(c4_net)
    for prec, bound in ((narvis.PRECISION_BF16, 2e-2), (narvis.PRECISION_FP8, 6e-2)):
        got = gpu_trained_forward(w, planes, prec)
        assert np.isfinite(got).all()
        errs = [float(np.abs(got[:, :, a:b, c:d] - wt).max()) for (a, b, c, d), wt in zip(tiles, wants)]
        print(f"  {'BF16' if prec == 0 else 'FP8'}: max |gpu - fp64| per tile {['%.4f' % e for e in errs]} "
              f"(bound {bound})", flush=True)
        assert max(errs) <= bound
