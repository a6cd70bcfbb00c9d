#!/usr/bin/env python3
"""Benchmark of the rasterizer hot path on one GPU.

One step = one frame of the whole path: host camera composition (FP64), key
clear, render (project + cull + 64-bit atomic-min visibility) and resolve
(depth, attribute planes and the colour channel; Vel2D too where the workload
has velocities).  Steps walk the workload's camera path.  Inputs are resident
in device memory before timing starts.

Prints one JSON line.  `value` is points rendered per second over the timed
steps; `roofline` reports the render kernel (the dominant one) against HBM
peak using HIP events recorded on the launch stream; `cpu_baseline` times the
CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpoints/s raster; 1080p frame ms raster+BF16 net vs Gaussian splat @PSNR"
HBM_PEAK_GBPS = 8000.0
RASTER_SRC = os.path.join(ROOT, "paper_2407_19097_amd", "csrc", "raster.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "render_traffic.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def make_scene(name, device):
    from paper_2407_19097_amd import scenes
    if name == "trajectories":
        return scenes.trajectories(device=device), "trajectories: 3.5M particles x 100 RK4 steps = 350M points, double gyre, 1920x1080, 120-frame fly-through + overview"
    if name == "vector_field":
        return scenes.vector_field(device=device), "vector field: 500x500x200 = 50M jittered points, Rankine vortex, 1920x1080, 60-frame orbit"
    if name == "unit_cube":
        sc = scenes.unit_cube()
        import torch
        sc.x, sc.y, sc.z = (torch.from_numpy(a).to(device) for a in (sc.x, sc.y, sc.z))
        sc.attrs = [torch.from_numpy(a).to(device) for a in sc.attrs]
        return sc, "unit cube: 1M points, 512x512"
    if name == "terrain":
        return scenes.terrain(device=device), "terrain: 1B jittered samples of an fBm height field, RGBA u8, 3840x2160"
    if name == "terrain25":
        sc = scenes.terrain(device=device)
        return scenes.subsample(sc, 4), "terrain, every 4th point: 250M points, 3840x2160"
    raise SystemExit(f"unknown workload {name}")


def read_traffic(launch_points, W, H):
    """HBM bytes per render launch from committed rocprofv3 counter runs, if
    they were taken on the current kernel source and the same workload."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256_16") != source_hash(RASTER_SRC):
        return None
    if rec.get("points") != launch_points or rec.get("W") != W or rec.get("H") != H:
        return None
    return rec.get("bytes_per_launch")


def host_cpu():
    """(threads this process may use, CPU model name)."""
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return max(1, cores), model


def cpu_baseline(sc, cams, budget_s=10.0):
    """The oracle as it stands on a bounded sample of the workload: the
    single-threaded C oracle on the first S points of frame 0, and its
    all-cores form (private key buffers merged by elementwise minimum, the
    same keys) on whole frames along the camera path; both followed by the
    oracle's resolve (depth and attribute planes)."""
    from oracle import camera as ocam
    from oracle import raster as orast
    n, W, H = sc.n, sc.W, sc.H
    cores, model = host_cpu()
    xs, ys, zs = (a.cpu().numpy() for a in (sc.x, sc.y, sc.z))
    attrs = []
    for a in sc.attrs:
        h = a.cpu().numpy()
        attrs.append(h.view(np.uint16) if h.dtype == np.int16 else h)
    M, near, far = ocam.clip_matrix(cams[0], W, H)
    # single thread: calibrate on 2M points, then the first S points
    cal = min(n, 2_000_000)
    t0 = time.perf_counter()
    orast.render(xs[:cal], ys[:cal], zs[:cal], M, near, far, W, H)
    rate = cal / max(time.perf_counter() - t0, 1e-6)
    S = int(min(n, max(cal, rate * budget_s)))
    t0 = time.perf_counter()
    keys = orast.render(xs[:S], ys[:S], zs[:S], M, near, far, W, H)
    orast.resolve(keys, W, H, xs, ys, zs, M, attrs)
    dt1 = time.perf_counter() - t0
    single = S / dt1 / 1e9
    # all cores: whole frames of the camera path within the budget
    t0 = time.perf_counter()
    keys = orast.render_mt(xs, ys, zs, M, near, far, W, H, cores)
    orast.resolve(keys, W, H, xs, ys, zs, M, attrs)
    first = time.perf_counter() - t0
    frames = max(1, min(len(cams) - 1, int(budget_s / max(first, 1e-6))))
    t0 = time.perf_counter()
    for f in range(1, 1 + frames) if len(cams) > 1 else range(frames):
        M, near, far = ocam.clip_matrix(cams[f % len(cams)], W, H)
        keys = orast.render_mt(xs, ys, zs, M, near, far, W, H, cores)
        orast.resolve(keys, W, H, xs, ys, zs, M, attrs)
    dtm = time.perf_counter() - t0
    del xs, ys, zs, attrs
    return {"value": frames * n / dtm / 1e9, "unit": "Gpoints/s", "cores": cores, "kind": "oracle",
            "cpu_model": model, "single_thread_value": round(single, 5),
            "sample": f"all-cores C oracle ({cores} threads, private key buffers merged by elementwise min), "
                      f"{frames} whole frame(s) of {n} points ({W}x{H}) along the camera path, render + resolve "
                      f"(depth, attributes), {dtm:.1f} s; single thread: first {S} points of frame 0, {dt1:.1f} s"}


def frame_section(torch, log_fn, frames=12, train_views=2000, train_steps=2500, unet_steps=1500):
    """1080p frame of the vector-field orbit: raster G-buffer + BF16 network
    vs the Gaussian splat.  The network and the paper's gated U-Net are first
    trained by the library's own kernels on the 9:1 training split of 2000
    hemisphere views at 512 x 512 (not timed)."""
    from paper_2407_19097_amd import metrics, narvis, scenes, train
    sc = scenes.vector_field(device="cuda")
    c4 = train.train_c4(sc, views=train_views, steps=train_steps, log=log_fn, unet_steps=unet_steps)
    u = c4.unet
    w, cal, heldout, train_s, losses = c4.weights, c4.cal, c4.heldout, c4.secs, c4.losses
    ntr = train_views - len(heldout)
    # training step throughput: 10 timed steps on a fixed batch of 16 views
    # (a separate, freshly initialised parameter set, so the trained one is
    # untouched); FLOPs counted as 3 x forward (forward, input gradients,
    # weight gradients)
    tw = narvis.NetWeights(train.init_blob(1))
    tws = torch.empty(narvis.narvis_train_workspace_size(16, 512, 512), dtype=torch.uint8, device="cuda")
    tl = torch.empty(1, dtype=torch.float32, device="cuda")
    fb = cal.contiguous()
    tb = torch.rand((16, 3, 512, 512), dtype=torch.float32, device="cuda")
    for _ in range(2):
        narvis.narvis_train_step(tw, fb, tb, 16, 512, 512, 1e-3, 1e-3, tl, tws)
    te0, te1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    te0.record()
    for _ in range(10):
        narvis.narvis_train_step(tw, fb, tb, 16, 512, 512, 1e-3, 1e-3, tl, tws)
    te1.record()
    torch.cuda.synchronize()
    train_step_ms = te0.elapsed_time(te1) / 10
    tw.close()
    del tws, tb
    # FP8: static activation scales calibrated on 16 training views
    cal_ws = torch.empty(narvis.narvis_train_workspace_size(16, 512, 512), dtype=torch.uint8, device="cuda")
    narvis.narvis_weights_calibrate_fp8(w, fb, 16, 512, 512, cal_ws)
    names = ["e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "e4a", "e4b", "d3a", "d3b", "d2a", "d2b", "d1a", "d1b", "head"]
    fp8_layers = [nm for i, nm in enumerate(names) if (narvis.narvis_weights_fp8_layers(w) >> i) & 1]
    del cal, fb, cal_ws
    W, H = 1920, 1080
    r = train.Renderer(sc, W, H)
    feat = torch.empty((1, 8, H * W), dtype=torch.float32, device="cuda")
    img = torch.empty((1, 3, H, W), dtype=torch.float32, device="cuda")
    tgt = torch.empty((3, H * W), dtype=torch.float32, device="cuda")
    ws = torch.empty(narvis.narvis_postprocess_workspace_size(1, W, H), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    picks = [int(k * len(sc.cameras) / frames) for k in range(frames)]
    t_r, t_n, t_s, p_net, p_ras, s_net, s_ras = [], [], [], [], [], [], []
    t_n8, p_net8 = [], []
    img8 = torch.empty_like(img)

    def timed(fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        fn()
        e1.record(stream)
        return e0, e1

    bf16 = lambda out: narvis.narvis_postprocess(w, feat, 1, W, H, out, ws, stream=stream)
    fp8 = lambda out: narvis.narvis_postprocess(w, feat, 1, W, H, out, ws, precision=narvis.PRECISION_FP8,
                                                stream=stream)
    uws = torch.empty(narvis.narvis_unet_workspace_size(u, 1, W, H), dtype=torch.uint8, device="cuda")
    uimg = torch.empty_like(img)
    unet = lambda out: narvis.narvis_unet_forward(u, feat, 1, W, H, out, uws, stream=stream)
    t_u, p_u, s_u = [], [], []
    # the frame loop as a viewer runs it (G-buffer, network, next frame), once
    # with the BF16 and once with the FP8 network; the first frame warms up
    for net, t_net in ((bf16, t_n), (fp8, t_n8), (unet, t_u)):
        evs = []
        for k in [picks[0]] + picks:
            evs.append((timed(lambda: r.gbuffer(sc.cameras[k], feat[0], hint=True)), timed(lambda: net(img))))
        torch.cuda.synchronize()
        for (g0, g1), (n0, n1) in evs[1:]:
            if net is bf16:
                t_r.append(g0.elapsed_time(g1))
            t_net.append(n0.elapsed_time(n1))
    # quality against the splat, and the splat's own time
    for rep, k in enumerate([picks[0]] + picks):
        cam = sc.cameras[k]
        r.gbuffer(cam, feat[0])
        bf16(img)
        fp8(img8)
        unet(uimg)
        sp = timed(lambda: r.splat(cam, tgt))
        torch.cuda.synchronize()
        if rep == 0:
            continue
        t_s.append(sp[0].elapsed_time(sp[1]))
        t3 = tgt.view(1, 3, H, W)
        y = img
        p_net8.append(metrics.psnr(img8, t3).item())
        p_u.append(metrics.psnr(uimg, t3).item())
        s_u.append(metrics.ssim(uimg, t3).item())
        p_net.append(metrics.psnr(y, t3).item())
        p_ras.append(metrics.psnr(feat[:, 0:3].view(1, 3, H, W), t3).item())
        s_net.append(metrics.ssim(y, t3).item())
        s_ras.append(metrics.ssim(feat[:, 0:3].view(1, 3, H, W), t3).item())
    pairs = narvis.narvis_splat_pair_count(r.ws, sc.n, W, H, r.params)  # of the last frame
    # the anisotropic target (Gaussians elongated along the velocity, s = 300,
    # the paper's stretch for its hurricane vector field) of the first frame
    del r
    torch.cuda.empty_cache()
    lut_t = torch.from_numpy(scenes.colour_lut()).cuda()
    inv = float(np.float32(1.0 / (sc.lut_max - sc.lut_min)))
    ap = narvis.SplatParams(sigma_px=1.5, opacity=1.0, color_mode=narvis.COLOR_LUT, color_attr=sc.lut_attr, lut=lut_t,
                            lut_min=sc.lut_min, lut_inv_range=inv, aniso=1, vel_attr=sc.vel_attr, stretch=300.0,
                            max_pairs=1)
    aws = torch.empty(narvis.narvis_splat_workspace_size(sc.n, W, H, ap), dtype=torch.uint8, device="cuda")
    cam0 = sc.cameras[picks[0]]
    apairs = narvis.narvis_splat_count_pairs((sc.x, sc.y, sc.z), sc.attrs, sc.n, cam0, W, H, ap, aws)
    del aws
    ap.max_pairs = apairs
    aws = torch.empty(narvis.narvis_splat_workspace_size(sc.n, W, H, ap), dtype=torch.uint8, device="cuda")
    aimg = lambda: narvis.narvis_splat((sc.x, sc.y, sc.z), sc.attrs, sc.n, cam0, W, H, tgt, ap, aws, stream=stream)
    aimg()
    ta = [timed(aimg) for _ in range(3)]
    torch.cuda.synchronize()
    aniso_ms = float(np.mean([a.elapsed_time(b) for a, b in ta]))
    del aws, uws
    w.close()
    u.close()
    m = lambda xs: float(np.mean(xs))
    raster_ms, net_ms, splat_ms = m(t_r), m(t_n), m(t_s)
    net_gflop = 327360.0 * W * H / 1e9
    return {"workload": "vector field 50M points, 1920x1080, 12 orbit frames (30 degrees apart; G-buffer by the bounded render with the previous frame's keys as hint); network trained on "
                        f"{ntr} 512x512 hemisphere views for {train_steps} Adam steps of batch 16 ({train_s:.0f} s, "
                        f"loss {losses[0][1]:.5f} -> {losses[-1][1]:.5f})",
            "raster_ms": round(raster_ms, 4), "net_bf16_ms": round(net_ms, 4),
            "frame_ms": round(raster_ms + net_ms, 4), "splat_ms": round(splat_ms, 3),
            "frame_fraction_of_splat": round((raster_ms + net_ms) / splat_ms, 4),
            "splat_pairs_last_frame": pairs, "splat_gpairs_per_s": round(pairs / (splat_ms / 1e3) / 1e9, 3),
            "psnr_db": round(m(p_net), 3), "ssim": round(m(s_net), 4),
            "psnr_raster_only_db": round(m(p_ras), 3), "ssim_raster_only": round(m(s_ras), 4),
            "train_step_ms_b16_512": round(train_step_ms, 3),
            "train_tflops": round(3 * 327360.0 * 512 * 512 * 16 / (train_step_ms / 1e3) / 1e12, 1),
            "net_tflops": round(net_gflop / net_ms, 2), "net_gflop_per_frame": round(net_gflop, 1),
            "net_fp8_ms": round(m(t_n8), 4), "frame_fp8_ms": round(raster_ms + m(t_n8), 4),
            "psnr_fp8_db": round(m(p_net8), 3), "fp8_layers": fp8_layers,
            "splat_aniso_ms": round(aniso_ms, 3), "splat_aniso_pairs": apairs,
            "splat_aniso": "Gaussians elongated along the velocity, s = 300, first frame",
            "unet": {"network": "the paper's gated U-Net, widths 64-128-256-512-1024, descriptors at 5 scales",
                     "train": f"{unet_steps} Adam steps of batch 16 on the same views ({c4.unet_secs:.0f} s, loss "
                              f"{c4.unet_losses[0][1]:.5f} -> {c4.unet_losses[-1][1]:.5f})",
                     "net_ms": round(m(t_u), 4), "frame_ms": round(raster_ms + m(t_u), 4),
                     "frame_fraction_of_splat": round((raster_ms + m(t_u)) / splat_ms, 4),
                     "tflops": round(unet_flop_per_px(narvis.UNET_WIDTHS) * W * 1088 / 1e12 / (m(t_u) / 1e3), 1),
                     "psnr_db": round(m(p_u), 3), "ssim": round(m(s_u), 4)}}


def splat_section(torch, log_fn, frames):
    """Isotropic (sigma 1.5 px) and anisotropic (s = 300) splats of `frames`
    vector-field orbit frames at 1920x1080, each timed with HIP events."""
    from paper_2407_19097_amd import narvis, scenes
    sc = scenes.vector_field(device="cuda")
    W, H = 1920, 1080
    lut = torch.from_numpy(scenes.colour_lut()).cuda()
    inv = float(np.float32(1.0 / (sc.lut_max - sc.lut_min)))
    img = torch.empty((3, W * H), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    cams = [sc.cameras[int(k * len(sc.cameras) / max(1, frames))] for k in range(max(1, frames))]
    out = {}
    for name, aniso in (("isotropic", 0), ("anisotropic_s300", 1)):
        p = narvis.SplatParams(sigma_px=1.5, opacity=1.0, color_mode=narvis.COLOR_LUT, color_attr=sc.lut_attr, lut=lut,
                               lut_min=sc.lut_min, lut_inv_range=inv, aniso=aniso, vel_attr=sc.vel_attr,
                               stretch=300.0, max_pairs=1 if aniso else 0)
        if aniso:
            ws = torch.empty(narvis.narvis_splat_workspace_size(sc.n, W, H, p), dtype=torch.uint8, device="cuda")
            p.max_pairs = max(narvis.narvis_splat_count_pairs((sc.x, sc.y, sc.z), sc.attrs, sc.n, c, W, H, p, ws)
                              for c in cams)
            del ws
        ws = torch.empty(narvis.narvis_splat_workspace_size(sc.n, W, H, p), dtype=torch.uint8, device="cuda")
        run = lambda c: narvis.narvis_splat((sc.x, sc.y, sc.z), sc.attrs, sc.n, c, W, H, img, p, ws, stream=stream)
        run(cams[0])
        ev = []
        for c in cams:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run(c)
            e1.record(stream)
            ev.append((e0, e1))
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        pairs = narvis.narvis_splat_pair_count(ws, sc.n, W, H, p)
        log_fn(f"{name}: {ms:.3f} ms per frame, {pairs} pairs in the last frame")
        out[name] = {"ms": round(ms, 3), "pairs_last_frame": pairs}
        del ws
        torch.cuda.empty_cache()
    return out


def unet_flop_per_px(widths):
    """Multiply-adds x 2 per pixel of the full-resolution grid, summed over the
    gated U-Net's convolutions (a level-l layer runs on 4^-l of the pixels)."""
    w = [int(v) for v in widths]
    f = 2.0 * 8 * 8                                                   # descriptors
    for l in range(5):
        f += 2.0 * 2 * w[l] * ((w[l - 1] if l else 8) + 8) * 9 / 4 ** l  # encoder
    for l in range(4):
        f += 2.0 * 4 * w[l] * w[l + 1] / 4 ** (l + 1)                   # transposed conv
        f += 2.0 * 2 * w[l] * 2 * w[l] * 9 / 4 ** l                     # decoder
    return f + 2.0 * 3 * w[0]                                         # head


def unet_section(torch, log_fn, frames=10):
    """The paper's gated U-Net (widths 64..1024, He-initialised): forward on
    one 1920x1080 frame (run on 1920x1088) and one training step of batch 16
    at 512x512, timed with HIP events."""
    from paper_2407_19097_amd import narvis, train
    widths = narvis.UNET_WIDTHS
    u = narvis.UNet(train.unet_init_blob(0, widths), widths)
    W, H = 1920, 1080
    stream = torch.cuda.current_stream()
    feat = torch.rand((1, 8, H, W), dtype=torch.float32, device="cuda")
    img = torch.empty((1, 3, H, W), dtype=torch.float32, device="cuda")
    ws = torch.empty(narvis.narvis_unet_workspace_size(u, 1, W, H), dtype=torch.uint8, device="cuda")
    fwd = lambda: narvis.narvis_unet_forward(u, feat, 1, W, H, img, ws, stream=stream)
    fwd()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(frames):
        fwd()
    e1.record(stream)
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / frames
    del ws, feat, img
    fpp = unet_flop_per_px(widths)
    gflop = fpp * W * 1088 / 1e9
    log_fn(f"gated U-Net forward 1920x1080: {fwd_ms:.3f} ms, {gflop:.0f} GFLOP, {gflop / fwd_ms:.1f} TFLOP/s")
    B, R = 16, 512
    tws = torch.empty(narvis.narvis_unet_workspace_size(u, B, R, R, train=True), dtype=torch.uint8, device="cuda")
    fb = torch.rand((B, 8, R, R), dtype=torch.float32, device="cuda")
    tb = torch.rand((B, 3, R, R), dtype=torch.float32, device="cuda")
    tl = torch.empty(1, dtype=torch.float32, device="cuda")
    step = lambda: narvis.narvis_unet_train_step(u, fb, tb, B, R, R, 1e-4, 1e-3, tl, tws, stream=stream)
    step()
    e0.record(stream)
    for _ in range(5):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / 5
    tflop = 3 * fpp * B * R * R / 1e12
    log_fn(f"gated U-Net training step b{B} {R}x{R}: {step_ms:.2f} ms, {tflop / (step_ms / 1e3):.1f} TFLOP/s")
    u.close()
    del tws, fb, tb
    torch.cuda.empty_cache()
    return {"widths": list(widths), "forward_1080p_ms": round(fwd_ms, 3), "gflop_per_frame": round(gflop, 1),
            "forward_tflops": round(gflop / fwd_ms, 1), "mflop_per_px": round(fpp / 1e6, 4),
            "train_step_ms_b16_512": round(step_ms, 2),
            "train_tflops": round(tflop / (step_ms / 1e3), 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=121)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="trajectories",
                    choices=["trajectories", "vector_field", "unit_cube", "terrain", "terrain25"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-frame", action="store_true", help="skip the 1080p raster+network vs splat frame section")
    ap.add_argument("--frame-only", action="store_true",
                    help="run only the 1080p frame section (for profiling the network kernels)")
    ap.add_argument("--train-steps", type=int, default=2500, help="Adam steps of the frame section's training")
    ap.add_argument("--unet-steps", type=int, default=1500, help="Adam steps of the frame section's U-Net training")
    ap.add_argument("--splat-only", action="store_true",
                    help="only time the Gaussian splat (isotropic and anisotropic) of vector-field frames at 1920x1080 "
                         "(for profiling the splat kernels)")
    ap.add_argument("--unet-only", action="store_true",
                    help="only time the paper's gated U-Net (forward at 1920x1080, a training step)")
    ap.add_argument("--no-layout", action="store_true",
                    help="skip the frames over the Morton layout (whole-batch culling)")
    ap.add_argument("--no-hinted", action="store_true",
                    help="skip the viewer loop with the previous frame's keys as hint (for profiling the plain stage)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the rasterizer runs on a single device "
              "(a multi-GPU run would shard points and min-reduce key buffers; not built)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2407_19097_amd import narvis, scenes

    if args.frame_only:
        print(json.dumps({"frame_1080p": frame_section(torch, log, train_steps=args.train_steps,
                                                       unet_steps=args.unet_steps)}), flush=True)
        return
    if args.unet_only:
        print(json.dumps({"unet": unet_section(torch, log)}), flush=True)
        return
    if args.splat_only:
        print(json.dumps({"splat_1080p": splat_section(torch, log, args.steps)}), flush=True)
        return

    dev = "cuda"
    t0 = time.time()
    sc, desc = make_scene(args.workload, dev)
    torch.cuda.synchronize()
    log(f"scene {sc.name}: {sc.n} points generated in {time.time() - t0:.1f}s")
    n, W, H = sc.n, sc.W, sc.H
    cams = sc.cameras
    mats = [narvis.narvis_camera_matrix(c, W, H) for c in cams]

    g = narvis.GBuffer.allocate(W, H, nattr=len(sc.attrs), depth=True, rgb=sc.lut_attr >= 0,
                                vel2d=sc.vel_attr >= 0)
    if sc.lut_attr >= 0:
        g.lut = torch.from_numpy(scenes.colour_lut()).to(dev)
        g.lut_attr, g.lut_min = sc.lut_attr, sc.lut_min
        g.lut_inv_range = float(np.float32(1.0 / (sc.lut_max - sc.lut_min)))
    g.vel_attr = sc.vel_attr
    pts = (sc.x, sc.y, sc.z)
    stream = torch.cuda.current_stream()

    def step(k, ev=None):
        # host camera composition is part of the step
        vp, nf, ff = narvis.narvis_camera_matrix(cams[k % len(cams)], W, H)
        narvis.narvis_raster_clear(g.keys, W, H, stream)
        if ev is not None:
            ev[0].record(stream)
        narvis.narvis_raster_render(pts, n, vp, nf, ff, W, H, g.keys, bounds=g.bounds, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        narvis.narvis_raster_resolve(pts, sc.attrs, n, vp, W, H, g, stream=stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    log("warmup done")

    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        step(k, evs[k])
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_host
    total_ms = start.elapsed_time(stop)
    render_ms = [a.elapsed_time(b) for a, b in evs]
    log(f"timed {args.steps} steps: {total_ms:.3f} ms on the stream, {wall * 1e3:.3f} ms wall")

    ms_per_step = total_ms / args.steps
    value = n * args.steps / (total_ms / 1e3) / 1e9
    render_avg = float(np.mean(render_ms))
    alg_bytes = 12.0 * n + 16.0 * W * H
    achieved = alg_bytes / (render_avg / 1e3) / 1e9
    traffic = read_traffic(n, W, H)

    # the same frames as a viewer loop that hands each render the previous
    # frame's keys as the hint of the bounded render (two key buffers in turn;
    # the result is the same bit for bit, checked on the last frame)
    def viewer_loop_hinted():
        log("viewer loop with the previous frame's keys as hint")
        bufs = [g.keys, torch.empty_like(g.keys)]

        def hinted_step(k, ev=None):
            vp, nf, ff = narvis.narvis_camera_matrix(cams[k % len(cams)], W, H)
            g.keys = bufs[k % 2]
            narvis.narvis_raster_clear(g.keys, W, H, stream)
            if ev is not None:
                ev[0].record(stream)
            narvis.narvis_raster_render(pts, n, vp, nf, ff, W, H, g.keys, bounds=g.bounds,
                                        hint_keys=bufs[(k + 1) % 2] if k > 0 else None, stream=stream)
            if ev is not None:
                ev[1].record(stream)
            narvis.narvis_raster_resolve(pts, sc.attrs, n, vp, W, H, g, stream=stream)

        for k in range(args.warmup):
            hinted_step(k)
        hevs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        start.record(stream)
        for k in range(args.steps):
            hinted_step(args.warmup + k, hevs[k])
        stop.record(stream)
        torch.cuda.synchronize()
        hinted_total = start.elapsed_time(stop)
        hinted_render = float(np.mean([a.elapsed_time(b) for a, b in hevs]))
        last = g.keys.clone()
        g.keys = bufs[0]
        vp, nf, ff = narvis.narvis_camera_matrix(cams[(args.warmup + args.steps - 1) % len(cams)], W, H)
        narvis.narvis_raster_clear(g.keys, W, H, stream)
        narvis.narvis_raster_render(pts, n, vp, nf, ff, W, H, g.keys, bounds=g.bounds, stream=stream)
        hinted_same = bool(torch.equal(g.keys, last))
        del bufs, last
        return {"value": round(n * args.steps / (hinted_total / 1e3) / 1e9, 3), "unit": "Gpoints/s",
                "ms_per_step": round(hinted_total / args.steps, 4), "render_stage_ms": round(hinted_render, 4),
                "hint": "previous frame's keys (hinted bounded render)",
                "same_keys_as_unhinted_last_frame": hinted_same}

    # (a moving camera only: with one view the hint would be the answer itself)
    hinted = None if args.no_hinted or len(cams) < 2 else viewer_loop_hinted()

    # the same frames rendered over the cloud's Morton layout (built once, not
    # timed per frame), whose batches are culled whole against the view volume
    # and the tile bounds; same keys bit for bit (checked on the last frame)
    def layout_loop():
        log("Morton layout: build, then the same frames with whole-batch culling")
        lb0, lb1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        lb0.record(stream)
        L = narvis.build_layout(pts, n)
        lb1.record(stream)
        torch.cuda.synchronize()
        build_ms = lb0.elapsed_time(lb1)

        def lstep(k, ev=None):
            vp, nf, ff = narvis.narvis_camera_matrix(cams[k % len(cams)], W, H)
            narvis.narvis_raster_clear(g.keys, W, H, stream)
            if ev is not None:
                ev[0].record(stream)
            narvis.narvis_raster_render_layout(L, n, vp, nf, ff, W, H, g.keys, bounds=g.bounds, stream=stream)
            if ev is not None:
                ev[1].record(stream)
            narvis.narvis_raster_resolve(pts, sc.attrs, n, vp, W, H, g, stream=stream)

        for k in range(args.warmup):
            lstep(k)
        levs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
        torch.cuda.synchronize()
        start.record(stream)
        for k in range(args.steps):
            lstep(k, levs[k])
        stop.record(stream)
        torch.cuda.synchronize()
        total = start.elapsed_time(stop)
        render = float(np.mean([a.elapsed_time(b) for a, b in levs]))
        last = g.keys.clone()
        vp, nf, ff = narvis.narvis_camera_matrix(cams[(args.steps - 1) % len(cams)], W, H)
        narvis.narvis_raster_clear(g.keys, W, H, stream)
        narvis.narvis_raster_render(pts, n, vp, nf, ff, W, H, g.keys, bounds=g.bounds, stream=stream)
        same = bool(torch.equal(g.keys, last))
        del L, last
        torch.cuda.empty_cache()
        saved = render_avg - render
        return {"value": round(n * args.steps / (total / 1e3) / 1e9, 3), "unit": "Gpoints/s",
                "ms_per_step": round(total / args.steps, 4), "render_stage_ms": round(render, 4),
                "layout_build_ms": round(build_ms, 2),
                "value_including_build": round(n * args.steps / ((total + build_ms) / 1e3) / 1e9, 3),
                "frames_to_repay_build": round(build_ms / saved, 1) if saved > 0 else None,
                "effective_frac": round(alg_bytes / (render / 1e3) / 1e9 / HBM_PEAK_GBPS, 4),
                "effective_frac_note": "algorithmic bytes of the whole cloud / render stage time / 8 TB/s; whole "
                                       "batches culled by their boxes are not read, so this is not HBM traffic",
                "layout": "stable sort by 30-bit Morton code, 2048-point batches with boxes; the depth sample "
                          "(every 8th point of that order) drawn first, then every batch; keys carry the "
                          "original index",
                "same_keys_as_original_order_last_frame": same}

    morton = None if args.no_layout else layout_loop()

    # coverage of the first frame, for context
    step(0)
    torch.cuda.synchronize()
    covered = float((g.keys != -1).float().mean().item())
    # fraction of the points inside the first frame's view volume (the rest
    # fail the frustum test), from plain torch arithmetic, for context
    m0 = [float(v) for v in mats[0][0]]
    visible = 0
    for s0 in range(0, n, 1 << 26):
        px, py, pz = sc.x[s0:s0 + (1 << 26)], sc.y[s0:s0 + (1 << 26)], sc.z[s0:s0 + (1 << 26)]
        w = ((px * m0[12] + py * m0[13]) + pz * m0[14]) + m0[15]
        sx = ((((px * m0[0] + py * m0[1]) + pz * m0[2]) + m0[3]) / w * 0.5 + 0.5) * W
        sy = (0.5 - (((px * m0[4] + py * m0[5]) + pz * m0[6]) + m0[7]) / w * 0.5) * H
        ok = (w >= float(mats[0][1])) & (w <= float(mats[0][2])) & (sx >= 0) & (sx < W) & (sy >= 0) & (sy < H)
        visible += int(ok.sum().item())
        del px, py, pz, w, sx, sy, ok

    # bandwidth of a plain streaming kernel (read 2 GiB, write 2 GiB), for
    # context and as the known-size reference for the HBM byte counters
    a = torch.ones(1 << 29, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    torch.abs(a, out=b)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        torch.abs(a, out=b)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_gbps = 5 * 2 * a.numel() * 4 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b

    # rate of random 64-bit atomic minima into a W x H buffer of int64 keys
    # (torch's scatter_reduce 'amin': one device-scope atomic per element), for
    # context beside the render's own atomics; the same kernel's L2 atomic
    # counter calibrates those counts
    m = 1 << 26
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    idx = torch.randint(0, W * H, (m,), device=dev, generator=gen)
    val = torch.randint(0, 1 << 62, (m,), device=dev, generator=gen)
    buf = torch.full((W * H,), (1 << 63) - 1, dtype=torch.int64, device=dev)
    buf.scatter_reduce_(0, idx, val, reduce="amin")
    atomic_ms = []
    for _ in range(3):
        buf.fill_((1 << 63) - 1)
        e0.record(stream)
        buf.scatter_reduce_(0, idx, val, reduce="amin")
        e1.record(stream)
        torch.cuda.synchronize()
        atomic_ms.append(e0.elapsed_time(e1))
    atomic_rate = m / (float(np.median(atomic_ms)) / 1e3)
    del idx, val, buf

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "points": n, "W": W, "H": H, "frames": len(cams),
                   "planes": ["keys", "depth"] + [f"attr:{nm}" for nm in sc.attr_names]
                   + (["rgb"] if sc.lut_attr >= 0 else []) + (["vel2d"] if sc.vel_attr >= 0 else []),
                   "covered_fraction_frame0": round(covered, 4),
                   "visible_point_fraction_frame0": round(visible / n, 4)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                     "kernel": "render stage: k_render_lds (every 8th chunk of 2048 points), k_tile_bounds, "
                               "k_render_cull (the other chunks against the bounds)",
                     "avg_launch_ms": round(render_avg, 4),
                     "algorithmic_bytes_per_launch": alg_bytes},
        "stream_copy_GBps": round(copy_gbps, 1),
        "atomic_min_u64_random_Gops": round(atomic_rate / 1e9, 3),
    }
    if hinted is not None:
        out["viewer_loop_hinted"] = hinted
    if morton is not None:
        out["morton_layout"] = morton
    if sc.name == "terrain" and W * H >= 3840 * 2160 and len(sc.attrs) >= 3:
        # end-to-end 4K frame: the whole-frame raster call resolves the RGB
        # (uint8 colours in the RGB8 mode) and depth planes straight into the
        # network's input tensor, then the BF16 network runs on it; the
        # velocity planes stay zero (the terrain has no velocity).  Untrained
        # weights: the network's time does not depend on them.
        log("end-to-end frame: raster into the network input, then the network")
        from paper_2407_19097_amd import train
        feat = torch.zeros((1, 8, W * H), dtype=torch.float32, device=dev)
        gf = narvis.GBuffer(keys=g.keys, depth=feat[0, 3], rgb=feat[0, 0:3], lut_attr=0,
                            rgb_mode=narvis.COLOR_RGB8, bounds=g.bounds)
        img = torch.empty((1, 3, H, W), dtype=torch.float32, device=dev)
        ws = torch.empty(narvis.narvis_postprocess_workspace_size(1, W, H), dtype=torch.uint8, device=dev)
        wts = narvis.NetWeights(train.init_blob(0))

        def e2e_frame(k):
            narvis.narvis_rasterize(pts, sc.attrs, n, cams[k % len(cams)], W, H, gf, stream=stream)
            narvis.narvis_postprocess(wts, feat, 1, W, H, img, ws, stream=stream)

        for k in range(2):
            e2e_frame(k)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for k in range(5):
            e2e_frame(k)
        e1.record(stream)
        e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e2.record(stream)
        for _ in range(5):
            narvis.narvis_postprocess(wts, feat, 1, W, H, img, ws, stream=stream)
        e3.record(stream)
        torch.cuda.synchronize()
        frame_ms = e0.elapsed_time(e1) / 5
        net_ms = e2.elapsed_time(e3) / 5
        wts.close()
        del feat, img, ws, gf
        out["end_to_end_frame"] = {"W": W, "H": H, "frame_ms": round(frame_ms, 4),
                                   "net_bf16_ms": round(net_ms, 4), "raster_ms": round(frame_ms - net_ms, 4),
                                   "net_tflops": round(327360.0 * W * H / (net_ms / 1e3) / 1e12, 1)}
    if not args.no_frame:
        log("1080p frame section: training the network, then raster + network vs splat")
        out["frame_1080p"] = frame_section(torch, log, train_steps=args.train_steps, unet_steps=args.unet_steps)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(sc, cams)
        out["cpu_baseline"]["value"] = round(out["cpu_baseline"]["value"], 5)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
