"""Oracle: the paper's cascaded MultiScale network and its SmallScale variant
(Sec. 3.1, Fig. 3) and its Unet (Sec. 3.1, Fig. 4), as the initial guess of
the pressure.  Plain FP64 (optionally emulating BF16 storage).  TEST
INFRASTRUCTURE ONLY.

What the paper fixes (Sec. 3.1 and the Fig. 3 caption): three scales of
n/4, n/2 and n pixels a side; the coarsest scale sees the input
interpolated onto the quarter-resolution mesh, its output is interpolated to
twice its size and concatenated with the input interpolated onto the
half-resolution mesh, which feeds the middle scale; the middle output is
interpolated to full size and concatenated with the full-resolution input,
which feeds the last scale.  5 layers at the coarsest scale, 7 at the other
two; kernels of 5x5, 3x3 and 1x1; ReLU after every convolution except the
last two of a branch; 418,640 parameters (SmallScale: the same structure
with about 1.3e5).

Readings where the paper is silent (its Fig. 3 with the widths is missing):

* every branch opens with a 5x5 convolution, ends with a 1x1 convolution to
  one channel, and has 3x3 convolutions in between;
* MultiScale widths: 64 channels everywhere, except the middle hidden layer
  of the two finer branches, which has 32 (419,459 parameters, +0.2 %);
  SmallScale: 32 channels everywhere (126,819 parameters);
* inputs and output as in the rest of this package: x = [d / s, solid],
  s = sqrt(mean_F d^2), phi0 = dx^2 s y_n on fluid cells (0 on solids);
  replicate padding;
* interpolation is bilinear with half-pixel centres and edge clamping (no
  anti-aliasing): to 1/2 size it is the 2x2 mean, to 1/4 size the mean of
  the central 2x2 pixels of every 4x4 block, to twice the size the usual
  9/16, 3/16, 3/16, 1/16 stencil.

Packed parameter layout (float32): branches from the coarsest (n/4) to the
finest (n); in each branch its layers in order, each as W[Cout][k][k][Cin]
then b[Cout].  Branch inputs: 2 channels at n/4; 3 channels (the two input
channels, then the upsampled coarser output) at n/2 and n.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from .cnn import bf16_round, up2

ARCHS = ("multiscale", "smallscale")

# Unet (Sec. 3.1, Fig. 4, whose widths are missing): five scales n .. n/16;
# per scale two 3x3 convolutions with ReLU on the way down, 2x2 max pooling
# between scales; on the way up, bilinear x2 upsampling, concatenation with
# the same scale's encoder output (skip first, then the upsampled map) and two
# 3x3 convolutions with ReLU; a linear 1x1 convolution to one channel.
# Widths (16, 16, 64, 64, 64) give 443,441 parameters (the paper: 443,521).
UNET_WIDTHS = (16, 16, 64, 64, 64)


def unet_layers():
    """(k, cin, cout, relu) in parameter order: encoder scales 0..4 (two
    layers each), decoder scales 3..0 (two layers each), output layer."""
    w = UNET_WIDTHS
    L, cin = [], 2
    for wl in w:
        L += [(3, cin, wl, True), (3, wl, wl, True)]
        cin = wl
    for l in range(len(w) - 2, -1, -1):
        L += [(3, w[l] + w[l + 1], w[l], True), (3, w[l], w[l], True)]
    L.append((1, w[0], 1, False))
    return L


def branches(arch: str):
    """Per branch (coarse to fine): list of (k, cin, cout, relu)."""
    if arch == "multiscale":
        a, mid = 64, 32
    elif arch == "smallscale":
        a, mid = 32, 32
    else:
        raise ValueError(arch)
    coarse = [(5, 2, a, True), (3, a, a, True), (3, a, a, True), (3, a, a, False),
              (1, a, 1, False)]
    finer = [(5, 3, a, True), (3, a, a, True), (3, a, mid, True), (3, mid, a, True),
             (3, a, a, True), (3, a, a, False), (1, a, 1, False)]
    return [coarse, finer, list(finer)]


def param_count(arch: str) -> int:
    if arch == "unet":
        return sum(k * k * ci * co + co for (k, ci, co, _r) in unet_layers())
    return sum(k * k * ci * co + co for br in branches(arch) for (k, ci, co, _r) in br)


def unpack(params: np.ndarray, arch: str):
    params = np.asarray(params, dtype=np.float64)
    assert params.size == param_count(arch), (params.size, param_count(arch))
    out, o = [], 0
    for br in branches(arch):
        layers = []
        for (k, ci, co, relu) in br:
            n = co * k * k * ci
            W = params[o:o + n].reshape(co, k, k, ci); o += n
            b = params[o:o + co]; o += co
            layers.append((W, b, relu))
        out.append(layers)
    return out


def conv_replicate(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """k x k convolution (k odd) with replicated edges:
    out[y, x, co] = b[co] + sum W[co, ky, kx, ci] xp[y + ky, x + kx, ci]."""
    H, Wd, cin = x.shape
    cout, k = W.shape[0], W.shape[1]
    h = k // 2
    xp = np.pad(x, ((h, h), (h, h), (0, 0)), mode="edge")
    cols = np.empty((H, Wd, k, k, cin))
    for ky in range(k):
        for kx in range(k):
            cols[:, :, ky, kx, :] = xp[ky:ky + H, kx:kx + Wd, :]
    return (cols.reshape(H * Wd, k * k * cin) @ W.reshape(cout, k * k * cin).T + b).reshape(H, Wd, cout)


def down(x: np.ndarray, f: int) -> np.ndarray:
    """Bilinear sampling to 1/f size with half-pixel centres: coarse pixel I
    samples the fine grid at (I + 0.5) f - 0.5 (clamped)."""
    def axis(n_fine):
        n = n_fine // f
        pos = np.clip((np.arange(n) + 0.5) * f - 0.5, 0.0, n_fine - 1)
        i0 = np.minimum(np.floor(pos).astype(np.int64), n_fine - 2)
        return i0, i0 + 1, pos - i0
    y0, y1, fy = axis(x.shape[0])
    x0, x1, fx = axis(x.shape[1])
    fy = fy[:, None, None]
    fx = fx[None, :, None]
    return ((1 - fy) * ((1 - fx) * x[np.ix_(y0, x0)] + fx * x[np.ix_(y0, x1)]) +
            fy * ((1 - fx) * x[np.ix_(y1, x0)] + fx * x[np.ix_(y1, x1)]))


def phi0(P: G.Plan, d: np.ndarray, dx: float, params, arch: str, bf16: bool = False):
    """Returns (phi0, s, ys) with ys the branch outputs (coarse to fine).
    ``bf16`` rounds the weights of the k > 1 layers, each such layer's input
    and each hidden layer's output to bfloat16 (the GPU's storage points);
    the 1x1 output layer reads the rounded activations with FP64 weights;
    accumulation stays FP64."""
    ny, nx = P.shape
    assert ny % 4 == 0 and nx % 4 == 0
    nets = unpack(params, arch)
    sumsq = float(np.sum(np.where(P.fluid, d, 0.0) ** 2))
    s = np.sqrt(sumsq / P.nF) if P.nF > 0 else 0.0
    if s == 0.0:
        return np.zeros(P.shape), 0.0, []
    x = np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)], axis=-1)
    rnd = bf16_round if bf16 else (lambda a: a)
    inputs = [down(x, 4), down(x, 2), x]
    ys, y = [], None
    for b, layers in enumerate(nets):
        h = inputs[b]
        if y is not None:
            h = np.concatenate([h, up2(y)[:, :, None]], axis=-1)
        for (W, bias, relu) in layers:
            if W.shape[1] == 1:  # 1x1 output layer: FP32 weights on the GPU
                h = conv_replicate(h, W, bias)
            else:
                h = conv_replicate(rnd(h), rnd(W), bias)
            if relu:
                h = np.maximum(h, 0.0)
            if W.shape[0] > 1:
                h = rnd(h)
        y = h[:, :, 0]
        ys.append(y)
    return np.where(P.fluid, dx * dx * s * y, 0.0), s, ys


def maxpool2(x: np.ndarray) -> np.ndarray:
    """2x2 max pooling, stride 2."""
    return np.maximum(np.maximum(x[0::2, 0::2], x[1::2, 0::2]), np.maximum(x[0::2, 1::2], x[1::2, 1::2]))


def up2c(t: np.ndarray) -> np.ndarray:
    """Bilinear x2 of every channel of an (H, W, C) map (as ``up2``)."""
    return np.stack([up2(t[:, :, c]) for c in range(t.shape[2])], axis=-1)


def unet_phi0(P: G.Plan, d: np.ndarray, dx: float, params, bf16: bool = False):
    """Returns (phi0, s).  ``bf16`` rounds the 3x3 weights, each 3x3 layer's
    input and output to bfloat16 (the GPU's storage points); max pooling and
    upsampling act on stored (rounded) maps and their results are stored
    again; the 1x1 output layer has FP64 weights."""
    ny, nx = P.shape
    assert ny % 16 == 0 and nx % 16 == 0
    params = np.asarray(params, dtype=np.float64)
    assert params.size == param_count("unet")
    layers, o = [], 0
    for (k, ci, co, relu) in unet_layers():
        W = params[o:o + co * k * k * ci].reshape(co, k, k, ci); o += co * k * k * ci
        b = params[o:o + co]; o += co
        layers.append((W, b, relu))
    sumsq = float(np.sum(np.where(P.fluid, d, 0.0) ** 2))
    s = np.sqrt(sumsq / P.nF) if P.nF > 0 else 0.0
    if s == 0.0:
        return np.zeros(P.shape), 0.0
    rnd = bf16_round if bf16 else (lambda a: a)

    def conv(h, i):
        W, b, relu = layers[i]
        out = conv_replicate(rnd(h), rnd(W), b)
        return rnd(np.maximum(out, 0.0) if relu else out)

    h = np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)], axis=-1)
    skips, li = [], 0
    nlev = len(UNET_WIDTHS)
    for lev in range(nlev):
        h = conv(conv(h, li), li + 1)
        li += 2
        if lev < nlev - 1:
            skips.append(h)
            h = maxpool2(h)
    for lev in range(nlev - 2, -1, -1):
        h = np.concatenate([skips[lev], rnd(up2c(h))], axis=-1)
        h = conv(conv(h, li), li + 1)
        li += 2
    W, b, _ = layers[li]
    y = conv_replicate(h, W, b)[:, :, 0]
    return np.where(P.fluid, dx * dx * s * y, 0.0), s
