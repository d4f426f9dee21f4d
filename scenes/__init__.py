"""Seeded synthetic inputs for the plume pressure-projection workloads.

This package draws random numbers and rasterises geometry into the input
flag mask; it holds none of the projection's arithmetic.  The CPU oracle and
the GPU library receive the arrays it returns unchanged, so both sides see
bit-identical inputs.

Workload recipe (paper Sec. 2.1 plume case, with the unit-square reading):

* unit square, ``nx`` x ``ny`` cells, ``dx = 1/nx``;
* walls on the left, right and bottom, open top;
* a bottom-centred inflow of width ``w`` (default 0.16 L) injecting light
  fluid at ``U_in = 1`` with density contrast ``drho`` (= Delta rho / rho0);
* gravity from the Richardson number, Eq. (1), with the inflow half-width as
  the length scale: ``g = Ri * U_in**2 / (drho * w/2)``;
* 0..3 disk obstacles, radius ~ U(0.05, 0.15) L, centre ~ U(0.2, 0.8) L per
  axis, a cell is solid when its centre lies strictly inside a disk;
* inflow-velocity noise ~ U(-1 %, +1 %) per inflow face per time step.

Random draws come from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order: number of obstacles, then each obstacle's (r, cx, cy), then the
density ratio when it is drawn.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

FLAG_SOLID = 1
FLAG_INFLOW = 2


@dataclass
class Scene:
    nx: int
    ny: int
    dx: float
    flags: np.ndarray  # (ny, nx) uint8: bit0 solid, bit1 "face below is inflow"
    disks: list = field(default_factory=list)  # [(r, cx, cy)] in domain units
    inflow_width: float = 0.16
    u_in: float = 1.0
    drho: float = 0.01
    ri: float = 0.1
    g: float = 125.0
    rho0: float = 1.0
    seed: int = 0


def rasterize(nx: int, ny: int, dx: float, disks, inflow_width: float) -> np.ndarray:
    """Input flag mask: solid cells of the disks and the inflow cells of row 0."""
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(x, y)
    solid = np.zeros((ny, nx), dtype=bool)
    for (r, cx, cy) in disks:
        solid |= (X - cx) ** 2 + (Y - cy) ** 2 < r * r
    flags = solid.astype(np.uint8) * FLAG_SOLID
    L = nx * dx
    inflow_cols = np.abs(x - 0.5 * L) < 0.5 * inflow_width
    flags[0, inflow_cols] |= FLAG_INFLOW
    return flags


def gravity_from_richardson(ri: float, u_in: float, drho: float, inflow_width: float) -> float:
    """Eq. (1) solved for g, with the inflow half-width as the length."""
    if ri == 0.0:
        return 0.0
    return ri * u_in * u_in / (drho * 0.5 * inflow_width)


def draw_disks(rng: np.random.Generator, n_obstacles: int, L: float = 1.0):
    disks = []
    for _ in range(n_obstacles):
        r = rng.uniform(0.05, 0.15) * L
        cx = rng.uniform(0.2, 0.8) * L
        cy = rng.uniform(0.2, 0.8) * L
        disks.append((float(r), float(cx), float(cy)))
    return disks


def plume_scene(n: int, seed: int = 0, n_obstacles=0, ny: int | None = None,
                inflow_width: float = 0.16, drho=0.01, ri: float = 0.1,
                u_in: float = 1.0, rho0: float = 1.0) -> Scene:
    """One plume scene.  ``n_obstacles`` is an int or a (lo, hi) inclusive range;
    ``drho`` is a float or a (lo, hi) range drawn uniformly."""
    rng = np.random.Generator(np.random.PCG64(seed))
    nx = n
    ny = n if ny is None else ny
    dx = 1.0 / nx
    if isinstance(n_obstacles, tuple):
        k = int(rng.integers(n_obstacles[0], n_obstacles[1] + 1))
    else:
        k = int(n_obstacles)
    disks = draw_disks(rng, k, L=1.0)
    if isinstance(drho, tuple):
        drho_v = float(rng.uniform(drho[0], drho[1]))
    else:
        drho_v = float(drho)
    flags = rasterize(nx, ny, dx, disks, inflow_width)
    g = gravity_from_richardson(ri, u_in, drho_v, inflow_width)
    return Scene(nx=nx, ny=ny, dx=dx, flags=flags, disks=disks,
                 inflow_width=inflow_width, u_in=u_in, drho=drho_v, ri=ri,
                 g=g, rho0=rho0, seed=seed)


def inflow_noise(seed: int, step: int, nx: int, amplitude: float = 0.01) -> np.ndarray:
    """Per-column inflow noise xi ~ U(-a, a) for one time step (float64).

    Each step draws from its own child stream, so any step can be
    regenerated without replaying the earlier ones."""
    ss = np.random.SeedSequence([seed, 7919, step])
    rng = np.random.Generator(np.random.PCG64(ss))
    return rng.uniform(-amplitude, amplitude, size=nx)


def random_faces(nx: int, ny: int, seed: int, kind: str = "smooth", modes: int = 6):
    """Random MAC face velocities u (ny, nx+1) and v (ny+1, nx), float64.

    ``smooth``: a sum of a few random low Fourier modes; ``white``: U(-1, 1)
    i.i.d.; ``mixed``: smooth plus 5 % white noise."""
    rng = np.random.Generator(np.random.PCG64(seed))
    if kind == "white":
        return rng.uniform(-1, 1, (ny, nx + 1)), rng.uniform(-1, 1, (ny + 1, nx))

    def smooth(shape, ox, oy):
        H, W = shape
        xs = (np.arange(W) + ox) / nx
        ys = (np.arange(H) + oy) / nx
        X, Y = np.meshgrid(xs, ys)
        out = np.zeros(shape)
        for _ in range(modes):
            kx, ky = rng.integers(1, 5, size=2)
            ph = rng.uniform(0, 2 * np.pi, size=2)
            a = rng.uniform(-1, 1)
            out += a * np.sin(np.pi * kx * X + ph[0]) * np.sin(np.pi * ky * Y + ph[1])
        return out

    u = smooth((ny, nx + 1), 0.0, 0.5)
    v = smooth((ny + 1, nx), 0.5, 0.0)
    if kind == "mixed":
        u = u + 0.05 * rng.uniform(-1, 1, u.shape)
        v = v + 0.05 * rng.uniform(-1, 1, v.shape)
    return u, v


def random_density(nx: int, ny: int, seed: int, rho0: float, drho: float, blobs: int = 4):
    """A smooth random density field (ny, nx), float64, between rho0 (1 - drho)
    and rho0: a few Gaussian blobs of lighter fluid (the plume's own density
    range) at random positions and widths."""
    rng = np.random.Generator(np.random.PCG64([seed, 104729]))
    X, Y = np.meshgrid((np.arange(nx) + 0.5) / nx, (np.arange(ny) + 0.5) / nx)
    light = np.zeros((ny, nx))
    for _ in range(blobs):
        cx, cy = rng.uniform(0.1, 0.9), rng.uniform(0.1, 0.9) * ny / nx
        w = rng.uniform(0.05, 0.2)
        light = np.maximum(light, rng.uniform(0.3, 1.0) * np.exp(-((X - cx) ** 2 + (Y - cy) ** 2) / (w * w)))
    return rho0 * (1.0 - drho * light)

# ---- network parameters -------------------------------------------------------

def cnn_param_count(scales: int, channels: int) -> int:
    """Parameters of the multi-scale net: per scale 4 conv3x3 (2->C, then C->C)
    with biases and a 1x1 C->1 output with bias."""
    C = channels
    per = (C * 9 * 2 + C) + 3 * (C * 9 * C + C) + (C + 1)
    return scales * per


def random_weights(scales: int, channels: int, seed: int, out_scale: float = 1.0) -> np.ndarray:
    """He-uniform random init in the packed float32 layout.

    Layout, for each scale s = 0 (finest) .. S-1: four 3x3 layers, each as
    weights [Cout][3][3][Cin] followed by bias [Cout] (Cin = 2 for the first
    layer, C after), then the 1x1 output as weights [C] and bias [1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    C = channels
    parts = []
    for _s in range(scales):
        cin = 2
        for _l in range(4):
            fan_in = 9 * cin
            bw = np.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-bw, bw, C * 9 * cin))
            parts.append(rng.uniform(-1, 1, C) / np.sqrt(fan_in))
            cin = C
        bo = out_scale / np.sqrt(C)
        parts.append(rng.uniform(-bo, bo, C))
        parts.append(np.zeros(1))
    w = np.concatenate(parts).astype(np.float32)
    assert w.size == cnn_param_count(scales, channels)
    return w


def zero_weights(scales: int, channels: int) -> np.ndarray:
    return np.zeros(cnn_param_count(scales, channels), dtype=np.float32)


# Layer shapes of the cascaded MultiScale / SmallScale networks, (k, cin, cout)
# per layer, branches from the coarsest to the finest (used only to size the
# random initialisation below).
def paper_net_layers(arch: str):
    if arch == "unet":  # one "branch": encoder, decoder, output layer
        w = (16, 16, 64, 64, 64)
        L, cin = [], 2
        for wl in w:
            L += [(3, cin, wl), (3, wl, wl)]
            cin = wl
        for l in range(3, -1, -1):
            L += [(3, w[l] + w[l + 1], w[l]), (3, w[l], w[l])]
        return [L + [(1, w[0], 1)]]
    a, mid = {"multiscale": (64, 32), "smallscale": (32, 32)}[arch]
    coarse = [(5, 2, a), (3, a, a), (3, a, a), (3, a, a), (1, a, 1)]
    finer = [(5, 3, a), (3, a, a), (3, a, mid), (3, mid, a), (3, a, a), (3, a, a), (1, a, 1)]
    return [coarse, finer, finer]


def random_paper_weights(arch: str, seed: int, out_scale: float = 1.0) -> np.ndarray:
    """He-uniform random init of a cascaded network in its packed float32
    layout: per layer W[Cout][k][k][Cin] then b[Cout], branches coarse to
    fine.  The output layers are scaled by ``out_scale``."""
    rng = np.random.Generator(np.random.PCG64([seed, 31337]))
    parts = []
    for br in paper_net_layers(arch):
        for i, (k, ci, co) in enumerate(br):
            fan_in = k * k * ci
            bw = np.sqrt(6.0 / fan_in) * (out_scale if i == len(br) - 1 else 1.0)
            parts.append(rng.uniform(-bw, bw, co * k * k * ci))
            parts.append(rng.uniform(-1, 1, co) / np.sqrt(fan_in))
    return np.concatenate(parts).astype(np.float32)
