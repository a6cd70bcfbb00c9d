"""Seeded synthetic point-cloud workloads and camera paths.

This module only manufactures inputs: point positions, per-point attributes,
camera placements (eye/target/up/fov/near/far, never a matrix) and colour
look-up tables.  It holds none of the renderer's arithmetic, so the GPU path
and the CPU oracle can both consume what it produces.

The paper's datasets (a hurricane large-eddy simulation, GEOS storm
trajectories and a LiDAR terrain scan, Sec. 4.1) are not available; the
generators below produce inputs with the same structure:

* ``unit_cube``       -- uniform points in [0,1)^3 with N(0,1) velocities
                         (the small parity workload, 1 M points at 512x512).
* ``vector_field``    -- a jittered 500x500x200 lattice carrying an analytic
                         Rankine vortex (stands in for the vector-field volume).
* ``trajectories``    -- particles advected by RK4 through the time-dependent
                         double gyre (stands in for the trajectory data set).
* ``terrain``         -- jittered samples of an fBm height field with RGBA
                         colours (stands in for the photometric terrain scan).

Camera conventions follow the training setup of Sec. 3.3: vertical field of
view 60 degrees, near plane 0.1, far plane 2e5, z is height.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

FOVY_DEG = 60.0
ZNEAR = 0.1
ZFAR = 2.0e5

# attribute dtype codes, identical to the C ABI's enumeration
U8, U16, F16, F32 = 0, 1, 2, 3
DTYPE_OF = {np.dtype(np.uint8): U8, np.dtype(np.uint16): U16,
            np.dtype(np.float16): F16, np.dtype(np.float32): F32}


@dataclass
class Camera:
    """A pinhole camera placement.  Composition into a matrix is not done here."""
    eye: Sequence[float]
    target: Sequence[float]
    up: Sequence[float] = (0.0, 0.0, 1.0)
    fovy_deg: float = FOVY_DEG
    znear: float = ZNEAR
    zfar: float = ZFAR


@dataclass
class Scene:
    """Point positions (SoA float32) plus attribute planes and camera path.

    ``x, y, z`` and every entry of ``attrs`` are numpy arrays or torch tensors
    of length ``n`` (torch for the large generators so they can be built on
    the device that will render them).
    """
    name: str
    x: object
    y: object
    z: object
    attrs: List[object]
    attr_names: List[str]
    cameras: List[Camera]
    W: int
    H: int
    lut_attr: int = -1
    lut_min: float = 0.0
    lut_max: float = 1.0
    vel_attr: int = -1
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


# ----------------------------------------------------------------------------
# colour look-up table (the user transfer function of Sec. 3.2)
# ----------------------------------------------------------------------------

_RAMP = np.array([  # control points of a blue -> cyan -> yellow -> red ramp
    [0.00, 0.05, 0.05, 0.45],
    [0.30, 0.00, 0.65, 0.90],
    [0.60, 0.95, 0.90, 0.20],
    [1.00, 0.85, 0.10, 0.05],
], dtype=np.float64)


def colour_lut(entries: int = 256) -> np.ndarray:
    """A piecewise-linear colour ramp sampled at bin centres, float32 [entries][3]."""
    t = (np.arange(entries, dtype=np.float64) + 0.5) / entries
    out = np.empty((entries, 3), dtype=np.float64)
    for c in range(3):
        out[:, c] = np.interp(t, _RAMP[:, 0], _RAMP[:, c + 1])
    return out.astype(np.float32)


# ----------------------------------------------------------------------------
# small parity workload
# ----------------------------------------------------------------------------

def unit_cube(n: int = 1_000_000, seed: int = 0, W: int = 512, H: int = 512) -> Scene:
    """Uniform points in the unit cube, velocity ~ N(0,1)^3 and speed |v|.

    Four float32 attributes (vx, vy, vz, |v|).  Camera at (2,2,2) looking at
    the origin with +z up.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    xyz = rng.random((3, n), dtype=np.float32)
    v = rng.standard_normal((3, n), dtype=np.float32)
    with np.errstate(over="ignore"):
        s = np.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2]).astype(np.float32)
    cams = [Camera(eye=(2.0, 2.0, 2.0), target=(0.0, 0.0, 0.0))]
    return Scene("unit_cube", np.ascontiguousarray(xyz[0]), np.ascontiguousarray(xyz[1]),
                 np.ascontiguousarray(xyz[2]),
                 [np.ascontiguousarray(v[0]), np.ascontiguousarray(v[1]),
                  np.ascontiguousarray(v[2]), s],
                 ["vx", "vy", "vz", "speed"], cams, W, H,
                 lut_attr=3, lut_min=0.0, lut_max=3.5, vel_attr=0)


# ----------------------------------------------------------------------------
# large workloads (torch, built on the device that renders them)
# ----------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _uniform(gen, shape, device, lo, hi):
    torch = _torch()
    return torch.rand(shape, generator=gen, device=device, dtype=torch.float32) * (hi - lo) + lo


def orbit_cameras(frames: int, centre=(0.5, 0.5, 0.2), radius=1.5, height=0.75) -> List[Camera]:
    """Orbit around ``centre`` at a fixed radius and height above it."""
    cams = []
    for k in range(frames):
        phi = 2.0 * math.pi * k / frames
        eye = (centre[0] + radius * math.cos(phi), centre[1] + radius * math.sin(phi),
               centre[2] + height)
        cams.append(Camera(eye=eye, target=centre))
    return cams


def vector_field(device="cpu", nx=500, ny=500, nz=200, seed=2, frames=60,
                 W=1920, H=1080, core_radius=0.1) -> Scene:
    """Jittered lattice over [0,1]x[0,1]x[0,0.4] with a Rankine vortex.

    Cell size 0.002 for the default 500x500x200 lattice; each point is moved by
    U(-0.5, 0.5) cells per axis.  Index = (k*ny + j)*nx + i.  The vortex turns
    about the vertical axis through (0.5, 0.5): tangential speed r/R inside the
    core radius R and R/r outside, no vertical component.  Attributes are
    vx, vy, vz, speed in float16.
    """
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    cell = 1.0 / nx
    n = nx * ny * nz
    i = torch.arange(nx, device=device, dtype=torch.float32)
    j = torch.arange(ny, device=device, dtype=torch.float32)
    k = torch.arange(nz, device=device, dtype=torch.float32)
    gz, gy, gx = torch.meshgrid(k, j, i, indexing="ij")
    jit = _uniform(gen, (3, n), device, -0.5, 0.5)
    x = ((gx.reshape(-1) + 0.5 + jit[0]) * cell).contiguous()
    y = ((gy.reshape(-1) + 0.5 + jit[1]) * (1.0 / ny)).contiguous()
    z = ((gz.reshape(-1) + 0.5 + jit[2]) * (0.4 / nz)).contiguous()
    del gx, gy, gz, jit
    dx = x - 0.5
    dy = y - 0.5
    r = torch.sqrt(dx * dx + dy * dy)
    R = core_radius
    vt = torch.where(r <= R, r / R, R / torch.clamp(r, min=1e-30))
    inv_r = torch.where(r > 0, 1.0 / torch.clamp(r, min=1e-30), torch.zeros_like(r))
    vx = (-dy * inv_r * vt)
    vy = (dx * inv_r * vt)
    vz = torch.zeros_like(vx)
    speed = torch.sqrt(vx * vx + vy * vy)
    attrs = [a.to(torch.float16).contiguous() for a in (vx, vy, vz, speed)]
    del dx, dy, r, vt, inv_r, vx, vy, vz, speed
    return Scene("vector_field", x, y, z, attrs, ["vx", "vy", "vz", "speed"],
                 orbit_cameras(frames), W, H, lut_attr=3, lut_min=0.0, lut_max=1.0,
                 vel_attr=0)


def double_gyre_velocity(x, y, t, A=0.1, eps=0.25, omega=2.0 * math.pi / 10.0):
    """Velocity of the time-periodic double gyre (Shadden et al. 2005) on [0,2]x[0,1]."""
    torch = _torch()
    a = eps * math.sin(omega * t)
    b = 1.0 - 2.0 * eps * math.sin(omega * t)
    f = (a * x + b) * x
    dfdx = 2.0 * a * x + b
    u = -math.pi * A * torch.sin(math.pi * f) * torch.cos(math.pi * y)
    v = math.pi * A * torch.cos(math.pi * f) * torch.sin(math.pi * y) * dfdx
    return u, v


def trajectories(device="cpu", px=2500, py=1400, steps=100, seed=3, dt=0.1,
                 frames=120, W=1920, H=1080) -> Scene:
    """Particles seeded on a jittered px x py grid over [0,2]x[0,1], advected by RK4.

    Position k of every particle is stored (k = 0..steps-1), particle-major
    (index = particle*steps + k).  Height encodes time: z = 0.5*k/(steps-1).
    Attributes: the step number (uint16) and the speed at that point (float16).
    Cameras: a fly-through along x at fixed height, plus a last static
    overview that sees the whole domain.
    """
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    P = px * py
    gi = torch.arange(px, device=device, dtype=torch.float32)
    gj = torch.arange(py, device=device, dtype=torch.float32)
    gy, gx = torch.meshgrid(gj, gi, indexing="ij")
    jit = _uniform(gen, (2, P), device, -0.5, 0.5)
    px_ = ((gx.reshape(-1) + 0.5 + jit[0]) * (2.0 / px)).contiguous()
    py_ = ((gy.reshape(-1) + 0.5 + jit[1]) * (1.0 / py)).contiguous()
    del gx, gy, jit
    n = P * steps
    X = torch.empty((P, steps), device=device, dtype=torch.float32)
    Y = torch.empty((P, steps), device=device, dtype=torch.float32)
    Z = torch.empty((P, steps), device=device, dtype=torch.float32)
    STEP = torch.empty((P, steps), device=device, dtype=torch.int16)
    SPD = torch.empty((P, steps), device=device, dtype=torch.float16)
    t = 0.0
    xs, ys = px_, py_
    for k in range(steps):
        u, v = double_gyre_velocity(xs, ys, t)
        X[:, k] = xs
        Y[:, k] = ys
        Z[:, k] = 0.5 * k / max(steps - 1, 1)
        STEP[:, k] = k
        SPD[:, k] = torch.sqrt(u * u + v * v).to(torch.float16)
        if k + 1 == steps:
            break
        k1x, k1y = u, v
        k2x, k2y = double_gyre_velocity(xs + 0.5 * dt * k1x, ys + 0.5 * dt * k1y, t + 0.5 * dt)
        k3x, k3y = double_gyre_velocity(xs + 0.5 * dt * k2x, ys + 0.5 * dt * k2y, t + 0.5 * dt)
        k4x, k4y = double_gyre_velocity(xs + dt * k3x, ys + dt * k3y, t + dt)
        xs = xs + (dt / 6.0) * (k1x + 2.0 * k2x + 2.0 * k3x + k4x)
        ys = ys + (dt / 6.0) * (k1y + 2.0 * k2y + 2.0 * k3y + k4y)
        t += dt
    cams = []
    for k in range(frames):
        ex = -0.5 + 3.0 * k / max(frames - 1, 1)
        cams.append(Camera(eye=(ex, -0.8, 0.9), target=(ex + 0.5, 0.5, 0.25)))
    cams.append(Camera(eye=(1.0, -1.6, 1.6), target=(1.0, 0.5, 0.2)))  # overview
    step_u16 = STEP.reshape(-1).view(torch.uint16) if hasattr(torch, "uint16") else STEP.reshape(-1)
    return Scene("trajectories", X.reshape(-1), Y.reshape(-1), Z.reshape(-1),
                 [step_u16, SPD.reshape(-1)], ["step", "speed"], cams, W, H,
                 lut_attr=1, lut_min=0.0, lut_max=0.35, extra={"particles": P, "steps": steps})


def _hash_u32(v):
    """A 32-bit integer mixer (lowbias32 by C. Wellons) on int64 tensors."""
    v = v & 0xFFFFFFFF
    v = v ^ (v >> 16)
    v = (v * 0x7FEB352D) & 0xFFFFFFFF
    v = v ^ (v >> 15)
    v = (v * 0x846CA68B) & 0xFFFFFFFF
    v = v ^ (v >> 16)
    return v


def _value_noise(xq, yq, cells: int, seed: int):
    """Smoothstep-interpolated lattice noise in [0,1) with ``cells`` cells per unit."""
    torch = _torch()
    fx = xq * cells
    fy = yq * cells
    ix = torch.floor(fx)
    iy = torch.floor(fy)
    tx = fx - ix
    ty = fy - iy
    tx = tx * tx * (3.0 - 2.0 * tx)
    ty = ty * ty * (3.0 - 2.0 * ty)
    ix = ix.to(torch.int64)
    iy = iy.to(torch.int64)

    def corner(ox, oy):
        h = _hash_u32((ix + ox) * 73856093 ^ (iy + oy) * 19349663 ^ (seed * 83492791))
        return (h >> 8).to(torch.float32) * (1.0 / 16777216.0)

    c00, c10, c01, c11 = corner(0, 0), corner(1, 0), corner(0, 1), corner(1, 1)
    top = c00 + (c10 - c00) * tx
    bot = c01 + (c11 - c01) * tx
    return top + (bot - top) * ty


def terrain(device="cpu", grid=16384, lattice=31623, n=1_000_000_000, seed=5,
            W=3840, H=2160, octaves=8, zscale=0.15, row_block=1024) -> Scene:
    """fBm height field on a grid x grid lattice over [0,1]^2, sampled by jittered points.

    Points sit at jittered nodes of a ``lattice`` x ``lattice`` grid (row-major,
    truncated to ``n``); their height is bilinearly interpolated from the
    height field.  Colour is RGBA uint8 from a height ramp, A = 255.
    """
    torch = _torch()
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    hf = torch.empty((grid, grid), device=device, dtype=torch.float32)
    coords = (torch.arange(grid, device=device, dtype=torch.float32) + 0.5) / grid
    for r0 in range(0, grid, row_block):
        r1 = min(grid, r0 + row_block)
        yq = coords[r0:r1, None].expand(r1 - r0, grid)
        xq = coords[None, :].expand(r1 - r0, grid)
        acc = torch.zeros((r1 - r0, grid), device=device, dtype=torch.float32)
        amp, cells, norm = 1.0, 4, 0.0
        for o in range(octaves):
            acc += amp * _value_noise(xq, yq, cells, seed * 131 + o)
            norm += amp
            amp *= 0.5
            cells *= 2
        hf[r0:r1] = acc * (zscale / norm)
    n = min(n, lattice * lattice)
    x = torch.empty(n, device=device, dtype=torch.float32)
    y = torch.empty(n, device=device, dtype=torch.float32)
    z = torch.empty(n, device=device, dtype=torch.float32)
    rgba = torch.empty((n, 4), device=device, dtype=torch.uint8)
    lut = torch.from_numpy((colour_lut(256) * 255.0 + 0.5).astype(np.uint8)).to(device)
    chunk = 1 << 26
    for s0 in range(0, n, chunk):
        s1 = min(n, s0 + chunk)
        idx = torch.arange(s0, s1, device=device, dtype=torch.int64)
        row = (idx // lattice).to(torch.float32)
        col = (idx % lattice).to(torch.float32)
        jit = _uniform(gen, (2, s1 - s0), device, -0.5, 0.5)
        xs = torch.clamp((col + 0.5 + jit[0]) / lattice, 0.0, 1.0)
        ys = torch.clamp((row + 0.5 + jit[1]) / lattice, 0.0, 1.0)
        gxf = torch.clamp(xs * grid - 0.5, 0.0, grid - 1.0)
        gyf = torch.clamp(ys * grid - 0.5, 0.0, grid - 1.0)
        gx0 = torch.clamp(torch.floor(gxf).to(torch.int64), max=grid - 2)
        gy0 = torch.clamp(torch.floor(gyf).to(torch.int64), max=grid - 2)
        tx = gxf - gx0.to(torch.float32)
        ty = gyf - gy0.to(torch.float32)
        flat = hf.reshape(-1)
        h00 = flat[gy0 * grid + gx0]
        h10 = flat[gy0 * grid + gx0 + 1]
        h01 = flat[(gy0 + 1) * grid + gx0]
        h11 = flat[(gy0 + 1) * grid + gx0 + 1]
        zs = (h00 + (h10 - h00) * tx) + ((h01 + (h11 - h01) * tx) - (h00 + (h10 - h00) * tx)) * ty
        x[s0:s1] = xs
        y[s0:s1] = ys
        z[s0:s1] = zs
        q = torch.clamp((zs * (256.0 / zscale)).to(torch.int64), 0, 255)
        rgba[s0:s1, :3] = lut[q]
        rgba[s0:s1, 3] = 255
    del hf
    cams = [Camera(eye=(0.5, -0.3, 0.6), target=(0.5, 0.5, 0.0))]
    attrs = [rgba[:, c] for c in range(4)]  # strided views: AoS RGBA, stride 4 bytes
    return Scene("terrain", x, y, z, attrs, ["r", "g", "b", "a"], cams, W, H,
                 extra={"rgba": rgba})


def subsample(scene: Scene, every: int) -> Scene:
    """Keep every ``every``-th point (uniform sub-sampling of Sec. 4.4.2)."""
    sl = slice(0, None, every)

    def take(a):
        t = a[sl]
        return t.contiguous() if hasattr(t, "contiguous") else np.ascontiguousarray(t)

    return Scene(scene.name + f"/{every}", take(scene.x), take(scene.y), take(scene.z),
                 [take(a) for a in scene.attrs], list(scene.attr_names), scene.cameras,
                 scene.W, scene.H, scene.lut_attr, scene.lut_min, scene.lut_max,
                 scene.vel_attr, dict(scene.extra))
