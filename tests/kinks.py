"""ReLU kinks in parity tests of the CNN gradient (test helpers, CPU only).

Where a hidden pre-activation z lies within FP32 rounding of zero, the FP32
GPU network and the FP64 oracle can take different ReLU branches, and the
backward pass then differs locally by O(1) (the kink is a discrete decision,
Sec. 3.1's ReLU layers).  Two ways to compare the gradients anyway:

* ``ambiguous_units``: flag every pixel with a unit whose |z| is at most
  ``tau`` times A = (|W| * |h|) + |b| (the sum of absolute terms, which bounds
  the rounding error of z), and ``kink_free_faces`` masks out the faces whose
  gradient such a unit can reach (its receptive field at that scale, pushed
  through the pyramid and the divergence adjoint);
* ``linear_regime``: raise the hidden biases, layer by layer from the
  oracle's own forward pass, so that every unit is strictly active; the net
  is then linear in its input and no decision is close.
"""
from __future__ import annotations

import numpy as np
from scipy import ndimage

from oracle import cnn as CN
from oracle import grid as G


def _inputs(P, u, v, dx, S):
    d = G.divergence(P, *G.enforce_bc(P, u, v), dx)
    s = np.sqrt(np.sum(np.where(P.fluid, d, 0.0) ** 2) / P.nF)
    x = np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)], axis=-1)
    pyr = [x]
    for _ in range(S - 1):
        pyr.append(CN.down2(pyr[-1]))
    return pyr


def pre_activation_ratios(P, u, v, dx, params, S, C):
    """Per scale: the smallest |z| / A over the hidden units of each pixel."""
    nets = CN.unpack(params, S, C)
    pyr = _inputs(P, u, v, dx, S)
    out = []
    for k in range(S):
        h = pyr[k]
        rmin = np.full(h.shape[:2], np.inf)
        for (W, b) in nets[k]["layers"]:
            z = CN.conv3x3_replicate(h, W, b)
            A = CN.conv3x3_replicate(np.abs(h), np.abs(W), np.abs(b))
            rmin = np.minimum(rmin, (np.abs(z) / np.maximum(A, 1e-300)).min(axis=-1))
            h = np.maximum(z, 0.0)
        out.append(rmin)
    return out


def ambiguous_units(P, u, v, dx, params, S, C, tau):
    return [r <= tau for r in pre_activation_ratios(P, u, v, dx, params, S, C)]


def kink_free_faces(flagged, ny, nx, layers=4):
    """Face masks (u: ny x nx+1, v: ny+1 x nx) of the faces whose gradient
    no flagged unit can change."""
    bad = np.zeros((ny, nx), dtype=bool)
    for k, F in enumerate(flagged):
        if not F.any():
            continue
        M = ndimage.binary_dilation(F, structure=np.ones((2 * layers + 1, 2 * layers + 1), bool))
        bad |= np.repeat(np.repeat(M, 1 << k, axis=0), 1 << k, axis=1)
    bad = ndimage.binary_dilation(bad, structure=np.ones((3, 3), bool)) if bad.any() else bad
    ubad = np.zeros((ny, nx + 1), dtype=bool)
    ubad[:, :nx] |= bad
    ubad[:, 1:] |= bad
    vbad = np.zeros((ny + 1, nx), dtype=bool)
    vbad[:ny] |= bad
    vbad[1:] |= bad
    return ~ubad, ~vbad


def linear_regime(P, u, v, dx, params, S, C, margin=0.01):
    """Copy of `params` (FP32-representable) whose hidden biases make every
    unit's pre-activation at least `margin` * max A of its channel."""
    w = np.array(params, dtype=np.float64)
    nets = CN.unpack(w, S, C)   # views into w
    pyr = _inputs(P, u, v, dx, S)
    for k in range(S):
        h = pyr[k]
        for (W, b) in nets[k]["layers"]:
            z0 = CN.conv3x3_replicate(h, W, np.zeros_like(b))
            A0 = CN.conv3x3_replicate(np.abs(h), np.abs(W), np.zeros_like(b))
            nb = (-z0).reshape(-1, z0.shape[-1]).max(axis=0) + margin * A0.reshape(-1, z0.shape[-1]).max(axis=0)
            b[:] = np.asarray(np.maximum(nb, 0.0) + margin, dtype=np.float32)
            h = np.maximum(CN.conv3x3_replicate(h, W, b), 0.0)
    return w
