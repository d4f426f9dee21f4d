"""Oracle: gradient of the divergence loss through the hybrid projection with
the paper's cascaded MultiScale (or SmallScale) network as the initial guess
(Sec. 3.1, Fig. 3; the training loss of Sec. 3.2).  Plain FP64,
hand-derived reverse mode.  TEST INFRASTRUCTURE ONLY.

The loss is the one of adjoint.py with the cascade of papernets.phi0 in
place of the parallel multi-scale network:

    d    = D u,  s = sqrt(mean_F d^2),  x = [d/s, solid]
    y_0  = branch_0(down(x, 4)),  y_1 = branch_1([down(x, 2), up2(y_0)]),
    y_2  = branch_2([x, up2(y_1)]),  phi0 = dx^2 s y_2  (0 on solid cells)
    phi  = K Jacobi sweeps from phi0 (omega)
    loss = scale * sum_F (d - L phi)^2

The adjoints of the pieces: a k x k convolution with replicate padding (the
padding adjoint folds the ghost pixels onto the edge pixels; k = 1, 3, 5),
ReLU (a mask of the layer's output), the bilinear down-sampling to 1/f size
(the transposed interpolation), the concatenation of the up-sampled coarser
output (the gradient of that channel goes back through the transposed
bilinear x2 to the coarser branch's output).  Only channel 0 of x depends on
the velocity (through d and s); the solid channel is constant.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import papernets as PN
from .adjoint import up2_T


def convk_backward(x: np.ndarray, W: np.ndarray, lam_out: np.ndarray):
    """Adjoint of papernets.conv_replicate (k x k, k odd) w.r.t. its input,
    weights and bias: returns (lam_x, dW, db)."""
    H, Wd, cin = x.shape
    cout, k = W.shape[0], W.shape[1]
    h = k // 2
    xp = np.pad(x, ((h, h), (h, h), (0, 0)), mode="edge")
    cols = np.empty((H, Wd, k, k, cin))
    for ky in range(k):
        for kx in range(k):
            cols[:, :, ky, kx, :] = xp[ky:ky + H, kx:kx + Wd, :]
    lam2 = lam_out.reshape(H * Wd, cout)
    dW = (lam2.T @ cols.reshape(H * Wd, k * k * cin)).reshape(cout, k, k, cin)
    db = lam2.sum(axis=0)
    lcols = (lam2 @ W.reshape(cout, k * k * cin)).reshape(H, Wd, k, k, cin)
    lxp = np.zeros((H + 2 * h, Wd + 2 * h, cin))
    for ky in range(k):
        for kx in range(k):
            lxp[ky:ky + H, kx:kx + Wd, :] += lcols[:, :, ky, kx, :]
    # padded index q reads x[clamp(q - h)]: fold the ghosts onto the edges
    lx = np.zeros_like(x)
    ry = np.clip(np.arange(H + 2 * h) - h, 0, H - 1)
    rx = np.clip(np.arange(Wd + 2 * h) - h, 0, Wd - 1)
    for qy in range(H + 2 * h):
        np.add.at(lx[ry[qy]], rx, lxp[qy])
    return lx, dW, db


def down_matrix(n_fine: int, f: int) -> np.ndarray:
    """The 1-D interpolation of papernets.down as a matrix (n_fine/f x
    n_fine): coarse pixel I samples the fine axis at (I + 0.5) f - 0.5."""
    n = n_fine // f
    M = np.zeros((n, n_fine))
    pos = np.clip((np.arange(n) + 0.5) * f - 0.5, 0.0, n_fine - 1)
    i0 = np.minimum(np.floor(pos).astype(np.int64), n_fine - 2)
    fr = pos - i0
    M[np.arange(n), i0] += 1.0 - fr
    M[np.arange(n), i0 + 1] += fr
    return M


def down_T(lam: np.ndarray, f: int, fine_shape) -> np.ndarray:
    """Adjoint of papernets.down(., f) for one channel."""
    My = down_matrix(fine_shape[0], f)
    Mx = down_matrix(fine_shape[1], f)
    return My.T @ lam @ Mx


def cascade_forward(P: G.Plan, d: np.ndarray, dx: float, params, arch: str):
    """phi0 (as papernets.phi0 without BF16) and what the reverse pass needs:
    every branch's input and every layer's input and output."""
    nets = PN.unpack(params, arch)
    fl = P.fluid
    s = float(np.sqrt(np.sum(np.where(fl, d, 0.0) ** 2) / P.nF)) if P.nF > 0 else 0.0
    if s == 0.0:
        return np.zeros(P.shape), dict(s=0.0)
    x = np.stack([np.where(fl, d / s, 0.0), (~fl).astype(np.float64)], axis=-1)
    inputs = [PN.down(x, 4), PN.down(x, 2), x]
    br, ys, y = [], [], None
    for b, layers in enumerate(nets):
        h = inputs[b]
        if y is not None:
            h = np.concatenate([h, PN.up2(y)[:, :, None]], axis=-1)
        ins, outs = [], []
        for (W, bias, relu) in layers:
            ins.append(h)
            h = PN.conv_replicate(h, W, bias)
            if relu:
                h = np.maximum(h, 0.0)
            outs.append(h)
        y = h[:, :, 0]
        ys.append(y)
        br.append(dict(ins=ins, outs=outs, layers=layers))
    phi0 = np.where(fl, dx * dx * s * y, 0.0)
    return phi0, dict(s=s, x=x, branches=br, ys=ys)


def loss_and_grad(flags, u, v, dx, params, arch, K, omega=1.0, scale=1.0):
    """Returns (loss, dL/du, dL/dv, dL/dparams) in FP64."""
    P = G.plan(flags)
    fl = P.fluid
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, dx)
    phi0, F = cascade_forward(P, d, dx, params, arch)
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
    s = F["s"]
    if s > 0.0:
        ys = F["ys"]
        lam_s = dx * dx * float(np.sum(lam_phi0 * ys[2]))
        lam_y = dx * dx * s * lam_phi0
        grads = []
        lam_x0 = np.zeros(P.shape)  # gradient of channel 0 of x = [d/s, solid]
        fine = P.shape
        for b in (2, 1, 0):
            B = F["branches"][b]
            layers, ins, outs = B["layers"], B["ins"], B["outs"]
            lam_h = lam_y[:, :, None]
            bgrads = [None] * len(layers)
            for i in range(len(layers) - 1, -1, -1):
                W, _bias, relu = layers[i]
                lam_pre = lam_h * (outs[i] > 0) if relu else lam_h
                lam_h, dW, db = convk_backward(ins[i], W, lam_pre)
                bgrads[i] = (dW, db)
            grads = bgrads + grads
            if b == 2:
                lam_x0 += lam_h[:, :, 0]
            else:
                lam_x0 += down_T(lam_h[:, :, 0], 4 if b == 0 else 2, fine)
            if b > 0:
                lam_y = up2_T(lam_h[:, :, 2])
        lam_x = np.where(fl, lam_x0, 0.0)
        lam_d = lam_d + lam_x / s
        lam_s -= float(np.sum(lam_x * d)) / (s * s)
        lam_d = lam_d + np.where(fl, lam_s * d / (P.nF * s), 0.0)
        dparams = np.concatenate([np.concatenate([g[0].ravel(), g[1]]) for g in grads])
    else:
        dparams = np.zeros(PN.param_count(arch))
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


def loss_only(flags, u, v, dx, params, arch, K, omega=1.0, scale=1.0) -> float:
    P = G.plan(flags)
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, dx)
    phi, _ = cascade_forward(P, d, dx, params, arch)
    kinv = np.where(P.fluid, 1.0 / np.maximum(P.k, 1.0), 0.0)
    for _ in range(K):
        phi = phi - omega * dx * dx * kinv * G.residual(P, d, phi, dx)
    r = G.residual(P, d, phi, dx)
    return scale * float(np.sum(r[P.fluid] ** 2))
