"""Training and evaluation driver of the learned post-process.

Training pairs follow Sec. 3.3 and the viewpoint strategy of the
supplementary material: views on a hemisphere around the point cloud's
bounding-box centre with radius 0.75 x the box diagonal, rendered at
512 x 512 with a 60 degree field of view; the input is the rasterizer's
RGB + depth + Vel2D G-buffer and the target is the Gaussian splat renderer's
image; 9:1 train/validation split; Adam, learning rate 1e-3, batch 16.
Every step runs in the library (narvis_rasterize, narvis_splat,
narvis_train_step, narvis_postprocess); this module only orchestrates.
"""
from __future__ import annotations

import math
import time
from typing import List, Optional

import numpy as np

from . import metrics, narvis, scenes


def hemisphere_views(n: int, centre, radius: float, seed: int, min_elev=0.08, max_elev=math.pi / 2 - 0.12) -> List[scenes.Camera]:
    """Random cameras on the upper hemisphere (azimuth uniform in [0, 2 pi),
    elevation uniform in [min_elev, max_elev]), looking at the centre."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = []
    for _ in range(n):
        th = rng.uniform(0.0, 2.0 * math.pi)
        ph = rng.uniform(min_elev, max_elev)
        eye = (centre[0] + radius * math.cos(ph) * math.cos(th), centre[1] + radius * math.cos(ph) * math.sin(th),
               centre[2] + radius * math.sin(ph))
        cams.append(scenes.Camera(eye=eye, target=tuple(centre)))
    return cams


class Renderer:
    """Rasterizer G-buffer planes and splat targets for one scene."""

    def __init__(self, sc: scenes.Scene, W: int, H: int, sigma=1.5, device="cuda"):
        import torch
        self.torch = torch
        self.sc, self.W, self.H = sc, W, H
        self.lut = torch.from_numpy(scenes.colour_lut()).to(device)
        self.inv = float(np.float32(1.0 / (sc.lut_max - sc.lut_min)))
        # two key buffers in turn, so that a frame can take the previous
        # frame's keys as the hint of its bounded render
        self.key_bufs = [torch.empty(W * H, dtype=torch.int64, device=device) for _ in range(2)]
        self.frame = 0
        self.bounds = narvis.raster_bounds(W, H, device)
        self.params = narvis.SplatParams(sigma_px=sigma, opacity=1.0, color_mode=narvis.COLOR_LUT,
                                         color_attr=sc.lut_attr, lut=self.lut, lut_min=sc.lut_min,
                                         lut_inv_range=self.inv)
        self.ws = torch.empty(max(1, narvis.narvis_splat_workspace_size(sc.n, W, H, self.params)), dtype=torch.uint8,
                              device=device)

    @property
    def keys(self):
        return self.key_bufs[self.frame % 2]

    def gbuffer(self, cam, out, hint=False):
        """out: float32 [8, H*W] view (r, g, b, depth, v'x, v'y, theta, |v'|).
        hint: the previous gbuffer() call's keys seed the bounded render (a
        viewer loop; the planes are the same either way)."""
        self.frame += 1
        g = narvis.GBuffer(keys=self.keys, depth=out[3], rgb=out[0:3], vel2d=out[4:8], lut=self.lut,
                           lut_attr=self.sc.lut_attr, lut_min=self.sc.lut_min, lut_inv_range=self.inv,
                           vel_attr=self.sc.vel_attr, bounds=self.bounds,
                           hint=self.key_bufs[(self.frame + 1) % 2] if hint else None)
        narvis.narvis_rasterize((self.sc.x, self.sc.y, self.sc.z), self.sc.attrs, self.sc.n, cam, self.W, self.H, g)

    def splat(self, cam, out):
        """out: float32 [3, H*W]."""
        narvis.narvis_splat((self.sc.x, self.sc.y, self.sc.z), self.sc.attrs, self.sc.n, cam, self.W, self.H, out,
                            self.params, self.ws)


def render_dataset(r: Renderer, cams, log=print):
    torch = r.torch
    n = len(cams)
    feats = torch.empty((n, 8, r.H * r.W), dtype=torch.float32, device="cuda")
    targets = torch.empty((n, 3, r.H * r.W), dtype=torch.float32, device="cuda")
    t0 = time.time()
    for i, cam in enumerate(cams):
        r.gbuffer(cam, feats[i])
        r.splat(cam, targets[i])
        if (i + 1) % 250 == 0:
            torch.cuda.synchronize()
            log(f"rendered {i + 1}/{n} views ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()
    return feats.view(n, 8, r.H, r.W), targets.view(n, 3, r.H, r.W)


def init_blob(seed: int) -> np.ndarray:
    """He-normal weights and zero biases in the library's blob order."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(8, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3), (64, 128, 3), (128, 128, 3), (128, 256, 3),
              (256, 256, 3), (384, 128, 3), (128, 128, 3), (192, 64, 3), (64, 64, 3), (96, 32, 3), (32, 32, 3),
              (32, 3, 1)]
    parts = []
    for ci, co, k in shapes:
        parts.append((rng.standard_normal(co * ci * k * k) * math.sqrt(2.0 / (ci * k * k))).astype(np.float32))
        parts.append(np.zeros(co, np.float32))
    blob = np.concatenate(parts)
    assert blob.size == narvis.narvis_net_param_count()
    return blob


def unet_init_blob(seed: int, widths=narvis.UNET_WIDTHS) -> np.ndarray:
    """He-normal weights (fan-in) and zero biases of the gated U-Net in the
    library's blob order: desc, enc0..enc4, (up_l, dec_l) for l = 3..0, head."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = [int(v) for v in widths]
    layers = [(8 * 8, 8, 8)]                                     # (weights, biases, fan-in)
    for l in range(5):
        cin = (w[l - 1] if l else 8) + 8
        layers.append((2 * w[l] * cin * 9, 2 * w[l], cin * 9))
    for l in (3, 2, 1, 0):
        layers.append((4 * w[l] * w[l + 1], w[l], w[l + 1]))
        layers.append((2 * w[l] * 2 * w[l] * 9, 2 * w[l], 2 * w[l] * 9))
    layers.append((3 * w[0], 3, w[0]))
    parts = []
    for nw, nb, fan in layers:
        parts.append((rng.standard_normal(nw) * math.sqrt(2.0 / fan)).astype(np.float32))
        parts.append(np.zeros(nb, np.float32))
    blob = np.concatenate(parts)
    assert blob.size == narvis.narvis_unet_param_count(widths)
    return blob


def train(weights, feats, targets, steps: int, batch=16, lr=1e-3, lam_tv=1e-3, seed=0,
          log=print, log_every=50, time_budget_s: Optional[float] = None):
    """Adam on random batches of (feats, targets); `weights` is a NetWeights
    (the small network) or a UNet (the paper's gated U-Net)."""
    import torch
    n, _, H, W = feats.shape
    unet = isinstance(weights, narvis.UNet)
    wsb = (narvis.narvis_unet_workspace_size(weights, batch, W, H, train=True) if unet
           else narvis.narvis_train_workspace_size(batch, W, H))
    step_fn = narvis.narvis_unet_train_step if unet else narvis.narvis_train_step
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    lossv = torch.empty(1, dtype=torch.float32, device="cuda")
    fb = torch.empty((batch, 8, H, W), dtype=torch.float32, device="cuda")
    tb = torch.empty((batch, 3, H, W), dtype=torch.float32, device="cuda")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    perm = torch.randperm(n, generator=gen, device="cuda")
    pos = 0
    losses = []
    t0 = time.time()
    for s in range(steps):
        if pos + batch > n:
            perm = torch.randperm(n, generator=gen, device="cuda")
            pos = 0
        idx = perm[pos:pos + batch]
        pos += batch
        torch.index_select(feats, 0, idx, out=fb)
        torch.index_select(targets, 0, idx, out=tb)
        step_fn(weights, fb, tb, batch, W, H, lr, lam_tv, lossv, ws)
        if (s + 1) % log_every == 0 or s + 1 == steps:
            l = float(lossv.item())
            losses.append((s + 1, l))
            log(f"step {s + 1}/{steps} loss {l:.5f} ({time.time() - t0:.1f}s)")
            if not math.isfinite(l):
                raise FloatingPointError("training loss is not finite")
        if time_budget_s is not None and time.time() - t0 > time_budget_s:
            torch.cuda.synchronize()
            log(f"time budget reached after {s + 1} steps")
            break
    torch.cuda.synchronize()
    return losses, time.time() - t0


C2_CENTRE = (0.5, 0.5, 0.2)
C2_DIAG = math.sqrt(1.0 + 1.0 + 0.4 * 0.4)


def c4_views(n: int = 2000, seed: int = 4) -> List[scenes.Camera]:
    """Hemisphere views of the vector-field volume (radius 0.75 x the box
    diagonal around the box centre); the last 10 % are held out."""
    return hemisphere_views(n, C2_CENTRE, 0.75 * C2_DIAG, seed=seed)


class C4:
    """What train_c4 returns: the trained small network (`weights`), 16
    training views' inputs for FP8 calibration (`cal`), the held-out cameras,
    training seconds and loss log, and, when asked for, the trained gated
    U-Net with its own seconds and loss log."""

    def __init__(self, **kw):
        self.__dict__.update(kw)


def train_c4(sc: scenes.Scene, views: int = 2000, steps: int = 2500, res: int = 512, seed: int = 0, log=print,
             unet_steps: int = 0, unet_lr: float = 1e-3) -> C4:
    """Train the post-process on the 9:1 training split of `views` hemisphere
    views of `sc` at res x res (G-buffer input, splat target), Adam lr 1e-3,
    batch 16, lam_tv 1e-3; with unet_steps > 0 the paper's gated U-Net is
    trained on the same views too (Adam lr unet_lr, batch 16)."""
    import torch
    cams = c4_views(views)
    ntr = int(0.9 * views)
    r = Renderer(sc, res, res)
    feats, targets = render_dataset(r, cams[:ntr], log=log)
    w = narvis.NetWeights(init_blob(seed))
    losses, secs = train(w, feats, targets, steps, batch=16, lr=1e-3, lam_tv=1e-3, seed=seed, log=log,
                         log_every=500)
    out = C4(weights=w, heldout=cams[ntr:], secs=secs, losses=losses, unet=None, unet_secs=0.0, unet_losses=[])
    if unet_steps > 0:
        u = narvis.UNet(unet_init_blob(seed))
        out.unet = u
        out.unet_losses, out.unet_secs = train(u, feats, targets, unet_steps, batch=16, lr=unet_lr, lam_tv=1e-3,
                                               seed=seed, log=log, log_every=250)
    out.cal = feats[:16].clone()
    del feats, targets, r
    torch.cuda.empty_cache()
    return out


def evaluate(weights, feats, targets, chunk=8):
    """(psnr of the network output, psnr of the raster's RGB planes alone, ssim net, ssim raster) vs targets;
    `weights` a NetWeights or a UNet."""
    import torch
    n, _, H, W = feats.shape
    unet = isinstance(weights, narvis.UNet)
    wsb = (narvis.narvis_unet_workspace_size(weights, chunk, W, H) if unet
           else narvis.narvis_postprocess_workspace_size(chunk, W, H))
    run = narvis.narvis_unet_forward if unet else narvis.narvis_postprocess
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    out = torch.empty((chunk, 3, H, W), dtype=torch.float32, device="cuda")
    p_net, p_ras, s_net, s_ras = [], [], [], []
    for i in range(0, n, chunk):
        b = min(chunk, n - i)
        run(weights, feats[i:i + b].contiguous(), b, W, H, out, ws)
        y = out[:b]
        t = targets[i:i + b]
        p_net.append(metrics.psnr(y, t))
        p_ras.append(metrics.psnr(feats[i:i + b, 0:3], t))
        s_net.append(metrics.ssim(y, t))
        s_ras.append(metrics.ssim(feats[i:i + b, 0:3], t))
    cat = lambda xs: torch.cat(xs).mean().item()
    return cat(p_net), cat(p_ras), cat(s_net), cat(s_ras)
