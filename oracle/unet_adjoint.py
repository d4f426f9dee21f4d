"""Oracle: gradient of the divergence loss through the hybrid projection with
the paper's Unet as the initial guess (Sec. 3.1, Fig. 4; the training loss
of Sec. 3.2).  Plain FP64, hand-derived reverse mode.  TEST INFRASTRUCTURE
ONLY.

The loss is the one of adjoint.py with the Unet in place of the parallel
multi-scale network:

    d    = D u,  s = sqrt(mean_F d^2),  x = [d/s, solid]
    phi0 = dx^2 s Unet(x; theta)           (0 on solid cells)
    phi  = K Jacobi sweeps from phi0 (omega)
    loss = scale * sum_F (d - L phi)^2

The Unet's pieces and their adjoints (the reading of papernets.py): 3x3
convolutions with replicate padding and ReLU (the padding adjoint folds the
ghost pixels onto the edge pixels), 2x2 max pooling (its adjoint routes a
window's gradient to the window element that attained the maximum; a tie
goes to the first in row-major order of the window), bilinear x2 upsampling
with half-pixel centres and edge clamp (its adjoint is the transposed
interpolation), concatenation with the skip connection (its adjoint splits
the gradient between the two inputs), and the linear 1x1 output layer.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import papernets as PN
from .adjoint import conv3x3_backward, up2_T


def maxpool2_argmax(x: np.ndarray):
    """Masks (H/2, W/2, C) of the window element that attains the maximum,
    in the window order (0,0), (0,1), (1,0), (1,1); ties to the first."""
    a, b, c, e = x[0::2, 0::2], x[0::2, 1::2], x[1::2, 0::2], x[1::2, 1::2]
    m = np.maximum(np.maximum(a, b), np.maximum(c, e))
    ia = a == m
    ib = (b == m) & ~ia
    ic = (c == m) & ~ia & ~ib
    ie = ~(ia | ib | ic)
    return ia, ib, ic, ie


def maxpool2_T(x: np.ndarray, lam: np.ndarray) -> np.ndarray:
    """Adjoint of 2x2 max pooling at x applied to lam (H/2, W/2, C)."""
    ia, ib, ic, ie = maxpool2_argmax(x)
    out = np.zeros_like(x)
    out[0::2, 0::2] = lam * ia
    out[0::2, 1::2] = lam * ib
    out[1::2, 0::2] = lam * ic
    out[1::2, 1::2] = lam * ie
    return out


def up2c_T(lam: np.ndarray) -> np.ndarray:
    """Adjoint of the channel-wise bilinear x2 (papernets.up2c)."""
    return np.stack([up2_T(lam[:, :, c]) for c in range(lam.shape[2])], axis=-1)


def _layers(params):
    params = np.asarray(params, dtype=np.float64)
    assert params.size == PN.param_count("unet")
    out, o = [], 0
    for (k, ci, co, relu) in PN.unet_layers():
        W = params[o:o + co * k * k * ci].reshape(co, k, k, ci); o += co * k * k * ci
        b = params[o:o + co]; o += co
        out.append((W, b, relu))
    return out


def unet_forward(P: G.Plan, d: np.ndarray, dx: float, params):
    """phi0 (as papernets.unet_phi0 without BF16) and what the reverse pass
    needs: every 3x3 layer's input and output, the skip maps, y and s."""
    layers = _layers(params)
    fl = P.fluid
    s = float(np.sqrt(np.sum(np.where(fl, d, 0.0) ** 2) / P.nF)) if P.nF > 0 else 0.0
    if s == 0.0:
        return np.zeros(P.shape), dict(s=0.0)
    h = np.stack([np.where(fl, d / s, 0.0), (~fl).astype(np.float64)], axis=-1)
    ins, outs, skips, li = [], [], [], 0
    nlev = len(PN.UNET_WIDTHS)

    def conv(h_, i):
        W, b, relu = layers[i]
        ins.append(h_)
        o = PN.conv_replicate(h_, W, b)
        o = np.maximum(o, 0.0) if relu else o
        outs.append(o)
        return o

    for lev in range(nlev):
        h = conv(conv(h, li), li + 1)
        li += 2
        if lev < nlev - 1:
            skips.append(h)
            h = PN.maxpool2(h)
    for lev in range(nlev - 2, -1, -1):
        h = np.concatenate([skips[lev], PN.up2c(h)], axis=-1)
        h = conv(conv(h, li), li + 1)
        li += 2
    W, b, _ = layers[li]
    y = PN.conv_replicate(h, W, b)[:, :, 0]
    phi0 = np.where(fl, dx * dx * s * y, 0.0)
    return phi0, dict(s=s, ins=ins, outs=outs, skips=skips, y=y, head_in=h, layers=layers)


def loss_and_grad(flags, u, v, dx, params, K, omega=1.0, scale=1.0):
    """Returns (loss, dL/du, dL/dv, dL/dparams) in FP64."""
    P = G.plan(flags)
    fl = P.fluid
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, dx)
    phi0, F = unet_forward(P, d, dx, params)
    kinv = np.where(fl, 1.0 / np.maximum(P.k, 1.0), 0.0)
    phi = phi0
    for _ in range(K):
        phi = phi - omega * dx * dx * kinv * G.residual(P, d, phi, dx)
    r = G.residual(P, d, phi, dx)
    loss = scale * float(np.sum(r[fl] ** 2))
    # the solver part, as adjoint.loss_and_grad
    lam_r = np.where(fl, 2.0 * scale * r, 0.0)
    lam_d = lam_r.copy()
    lam = -G.laplacian(P, lam_r, dx)
    for _ in range(K):
        mu = kinv * lam
        lam_d = lam_d - omega * dx * dx * mu
        lam = lam + omega * dx * dx * G.laplacian(P, mu, dx)
    lam_phi0 = np.where(fl, lam, 0.0)
    nparam = PN.param_count("unet")
    s = F["s"]
    if s > 0.0:
        layers = F["layers"]
        ins, outs, skips = F["ins"], F["outs"], F["skips"]
        grads = [None] * len(layers)
        lam_s = dx * dx * float(np.sum(lam_phi0 * F["y"]))
        lam_y = dx * dx * s * lam_phi0
        # 1x1 output layer
        Wo, _bo, _ = layers[-1]
        h = F["head_in"]
        grads[-1] = (np.einsum("yx,yxc->c", lam_y, h).reshape(Wo.shape), np.array([lam_y.sum()]))
        lam_h = lam_y[:, :, None] * Wo.reshape(1, 1, -1)
        nlev = len(PN.UNET_WIDTHS)
        wid = PN.UNET_WIDTHS
        lam_skip = [None] * (nlev - 1)
        li = len(layers) - 2  # last decoder 3x3 layer
        for lev in range(nlev - 1):  # decoder levels 0, 1, 2, 3 (reverse of the forward)
            for _ in range(2):
                W, _b, _r = layers[li]
                lam_pre = lam_h * (outs[li] > 0)
                lam_h, dW, db = conv3x3_backward(ins[li], W, lam_pre)
                grads[li] = (dW, db)
                li -= 1
            # lam_h is the gradient of the concatenation [skip, up(h below)]
            lam_skip[lev] = lam_h[:, :, :wid[lev]]
            lam_h = up2c_T(lam_h[:, :, wid[lev]:])
        for lev in range(nlev - 1, -1, -1):  # encoder levels 4 .. 0
            if lev < nlev - 1:
                lam_h = lam_h + lam_skip[lev]
            for _ in range(2):
                W, _b, _r = layers[li]
                lam_pre = lam_h * (outs[li] > 0)
                lam_h, dW, db = conv3x3_backward(ins[li], W, lam_pre)
                grads[li] = (dW, db)
                li -= 1
            if lev > 0:
                lam_h = maxpool2_T(skips[lev - 1], lam_h)
        assert li == -1
        lam_x = np.where(fl, lam_h[:, :, 0], 0.0)
        lam_d = lam_d + lam_x / s
        lam_s -= float(np.sum(lam_x * d)) / (s * s)
        lam_d = lam_d + np.where(fl, lam_s * d / (P.nF * s), 0.0)
        dparams = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    else:
        dparams = np.zeros(nparam)
    lam_d = np.where(fl, lam_d, 0.0)
    ny, nx = P.shape
    gu = np.zeros((ny, nx + 1))
    gv = np.zeros((ny + 1, nx))
    gu[:, 1:nx] = (lam_d[:, :-1] - lam_d[:, 1:]) / dx
    gv[1:ny, :] = (lam_d[:-1, :] - lam_d[1:, :]) / dx
    gv[ny, :] = lam_d[ny - 1, :] / dx
    gv[0, :] = -lam_d[0, :] / dx
    gu = np.where(P.uopen, gu, 0.0)
    gv[1:] = np.where(P.vopen[1:], gv[1:], 0.0)
    gv[0] = np.where(P.vinflow, gv[0], 0.0)
    return loss, gu, gv, dparams


def loss_only(flags, u, v, dx, params, K, omega=1.0, scale=1.0) -> float:
    P = G.plan(flags)
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, dx)
    phi, _ = unet_forward(P, d, dx, params)
    kinv = np.where(P.fluid, 1.0 / np.maximum(P.k, 1.0), 0.0)
    for _ in range(K):
        phi = phi - omega * dx * dx * kinv * G.residual(P, d, phi, dx)
    r = G.residual(P, d, phi, dx)
    return scale * float(np.sum(r[P.fluid] ** 2))
