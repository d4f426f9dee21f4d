"""Oracle: the paper's cascaded MultiScale network and its SmallScale variant
(Sec. 3.1, Fig. 3), as the initial guess of the pressure.  Plain FP64
(optionally emulating BF16 storage).  TEST INFRASTRUCTURE ONLY.

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
