"""Oracle: the multi-scale CNN initial guess for the pressure.  Plain FP64
(optionally emulating BF16 storage).  TEST INFRASTRUCTURE ONLY.

Architecture (the parallel-branch multi-scale net; Sec. 3.1 MultiScale idea:
several resolutions of the same input, bilinear down/up sampling,
replication padding, ReLU on the hidden layers, linear output):

* input at full resolution: x = [d / s, solid] with s = sqrt(mean_F d^2);
* pyramid: x_{k+1} = 2x2 mean of x_k (bilinear half-size sampling with
  half-pixel centres), k = 0..S-2;
* per scale k: 4 x [conv 3x3, replicate pad, bias, ReLU] with C channels,
  then a 1x1 conv C -> 1 with bias (no activation): y_k;
* combine coarse to fine: t = y_{S-1}; t = y_k + up2(t) for k = S-2..0,
  up2 = bilinear x2 with half-pixel centres and edge clamp;
* phi0 = dx^2 * s * t, set to 0 on solid cells.

Packed parameter layout (float32): for each scale k = 0..S-1, four 3x3
layers as W[Cout][3][3][Cin] then b[Cout] (Cin = 2 first, then C), followed
by the 1x1 output as w[C] then b[1].
"""
from __future__ import annotations

import numpy as np

from . import grid as G


def param_count(S: int, C: int) -> int:
    return S * ((C * 9 * 2 + C) + 3 * (C * 9 * C + C) + C + 1)


def unpack(params: np.ndarray, S: int, C: int):
    params = np.asarray(params, dtype=np.float64)
    assert params.size == param_count(S, C), (params.size, param_count(S, C))
    out = []
    o = 0
    for _k in range(S):
        layers = []
        cin = 2
        for _l in range(4):
            n = C * 9 * cin
            W = params[o:o + n].reshape(C, 3, 3, cin); o += n
            b = params[o:o + C]; o += C
            layers.append((W, b))
            cin = C
        wo = params[o:o + C]; o += C
        bo = float(params[o]); o += 1
        out.append(dict(layers=layers, wo=wo, bo=bo))
    return out


def bf16_round(x: np.ndarray) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64.  Goes through float32, whose upper 16 bits are a bfloat16."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    b = (b + 0x7FFF + lsb) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3_replicate(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """out[y, x, co] = b[co] + sum_{ky,kx,ci} W[co,ky,kx,ci] * xp[y+ky, x+kx, ci]
    where xp is x padded by one pixel with replicated edge values."""
    H, Wd, cin = x.shape
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)), mode="edge")
    cols = np.empty((H, Wd, 3, 3, cin))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, ky, kx, :] = xp[ky:ky + H, kx:kx + Wd, :]
    cout = W.shape[0]
    out = cols.reshape(H * Wd, 9 * cin) @ W.reshape(cout, 9 * cin).T + b
    return out.reshape(H, Wd, cout)


def down2(x: np.ndarray) -> np.ndarray:
    """2x2 mean (= bilinear sampling to half size with half-pixel centres)."""
    return 0.25 * (x[0::2, 0::2] + x[1::2, 0::2] + x[0::2, 1::2] + x[1::2, 1::2])


def up2(t: np.ndarray) -> np.ndarray:
    """Bilinear x2 with half-pixel centres: fine pixel J samples the coarse
    grid at (J + 0.5)/2 - 0.5, clamped to the coarse extent."""
    H, W = t.shape

    def axis(n_coarse):
        pos = (np.arange(2 * n_coarse) + 0.5) / 2.0 - 0.5
        pos = np.clip(pos, 0.0, n_coarse - 1)
        i0 = np.minimum(np.floor(pos).astype(np.int64), max(n_coarse - 2, 0))
        f = pos - i0
        i1 = np.minimum(i0 + 1, n_coarse - 1)
        return i0, i1, f

    y0, y1, fy = axis(H)
    x0, x1, fx = axis(W)
    a = t[np.ix_(y0, x0)]
    b_ = t[np.ix_(y0, x1)]
    c = t[np.ix_(y1, x0)]
    d = t[np.ix_(y1, x1)]
    fy = fy[:, None]
    fx = fx[None, :]
    return (1 - fy) * ((1 - fx) * a + fx * b_) + fy * ((1 - fx) * c + fx * d)


def cnn_phi0(P: G.Plan, d: np.ndarray, dx: float, params, S: int, C: int,
             bf16: bool = False, keep: bool = False):
    """Returns (phi0, s, cache).  ``bf16`` rounds the 3x3 weights, each 3x3
    layer's input and each 3x3 layer's output to bfloat16 (the GPU's storage
    points); accumulation stays FP64, the 1x1 output and phi0 stay FP64."""
    ny, nx = P.shape
    assert ny % (1 << (S - 1)) == 0 and nx % (1 << (S - 1)) == 0
    nets = unpack(params, S, C)
    sumsq = float(np.sum(np.where(P.fluid, d, 0.0) ** 2))
    s = np.sqrt(sumsq / P.nF) if P.nF > 0 else 0.0
    cache = dict(s=s)
    if s == 0.0:
        return np.zeros(P.shape), 0.0, cache
    x = np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)], axis=-1)
    pyr = [x]
    for _k in range(S - 1):
        pyr.append(down2(pyr[-1]))
    ys = []
    acts = []
    rnd = bf16_round if bf16 else (lambda a: a)
    for k in range(S):
        h = rnd(pyr[k])
        a_k = [h]
        for (W, b) in nets[k]["layers"]:
            h = np.maximum(conv3x3_replicate(h, rnd(W), b), 0.0)
            h = rnd(h)
            a_k.append(h)
        y = h @ nets[k]["wo"] + nets[k]["bo"]
        ys.append(y)
        acts.append(a_k)
    t = ys[S - 1]
    for k in range(S - 2, -1, -1):
        t = ys[k] + up2(t)
    phi0 = np.where(P.fluid, dx * dx * s * t, 0.0)
    if keep:
        cache.update(pyr=pyr, acts=acts, ys=ys, t=t)
    return phi0, s, cache
