"""Oracle: gradient of the divergence loss through the hybrid projection.
Plain FP64, hand-derived reverse mode.  TEST INFRASTRUCTURE ONLY.

Training loss of Sec. 3.2 (the physics-driven loss on the divergence of
the corrected velocity; the paper notes that the gradient of the correction,
Eq. 2, is known so that back-propagation goes through it):

    d    = D u                       (faces with the boundary faces enforced)
    s    = sqrt(mean_F d^2)
    phi0 = dx^2 s CNN([d/s, solid]; theta)       (0 on solid cells)
    phi  = K Jacobi sweeps from phi0 (omega)
    r    = d - L phi                 (= div(u - grad phi))
    loss = scale * sum_F r^2

Reverse sweep, with L symmetric on fluid cells and M = diag(1/k_c):
    lam_r = 2 scale r;  lam_phi = -L lam_r;  lam_d = lam_r
    per reversed sweep: mu = M lam_phi; lam_d -= omega dx^2 mu;
                        lam_phi += omega dx^2 L mu
    CNN: phi0 scaling, upsample-sum transpose, 1x1 and 3x3 layers
    (ReLU masks, replicate-padding adjoint folds ghost pixels onto the edge),
    2x2-mean pyramid transpose, the d/s normalisation incl. ds/dd
    faces: lam_u = D^T lam_d on open and inflow faces, 0 on closed faces.

long_term() adds the paper's long-term term: the same loss after n unrolled
time steps, with the advection not differentiated (Sec. 3.2, Fig. 5, Eq. 4).
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import cnn as CN
from . import advect as AD


def _axis_matrix(n_coarse: int) -> np.ndarray:
    """Interpolation matrix (2n x n) of one axis of up2 (half-pixel centres,
    clamp), the same sampling rule as cnn.up2."""
    Umat = np.zeros((2 * n_coarse, n_coarse))
    pos = np.clip((np.arange(2 * n_coarse) + 0.5) / 2.0 - 0.5, 0.0, n_coarse - 1)
    i0 = np.minimum(np.floor(pos).astype(np.int64), max(n_coarse - 2, 0))
    f = pos - i0
    i1 = np.minimum(i0 + 1, n_coarse - 1)
    for J in range(2 * n_coarse):
        Umat[J, i0[J]] += 1 - f[J]
        Umat[J, i1[J]] += f[J]
    return Umat


def up2_T(lam: np.ndarray) -> np.ndarray:
    H2, W2 = lam.shape
    Uy = _axis_matrix(H2 // 2)
    Ux = _axis_matrix(W2 // 2)
    return Uy.T @ lam @ Ux


def down2_T(lam: np.ndarray) -> np.ndarray:
    """Adjoint of the 2x2 mean: each fine pixel receives a quarter."""
    return 0.25 * np.repeat(np.repeat(lam, 2, axis=0), 2, axis=1)


def conv3x3_backward(x: np.ndarray, W: np.ndarray, lam_out: np.ndarray, need_input: bool = True):
    """Adjoint of conv3x3_replicate w.r.t. its input, weights and bias."""
    H, Wd, cin = x.shape
    cout = W.shape[0]
    xp = np.pad(x, ((1, 1), (1, 1), (0, 0)), mode="edge")
    cols = np.empty((H, Wd, 3, 3, cin))
    for ky in range(3):
        for kx in range(3):
            cols[:, :, ky, kx, :] = xp[ky:ky + H, kx:kx + Wd, :]
    lam2 = lam_out.reshape(H * Wd, cout)
    dW = (lam2.T @ cols.reshape(H * Wd, 9 * cin)).reshape(cout, 3, 3, cin)
    db = lam2.sum(axis=0)
    if not need_input:
        return None, dW, db
    lcols = (lam2 @ W.reshape(cout, 9 * cin)).reshape(H, Wd, 3, 3, cin)
    lxp = np.zeros((H + 2, Wd + 2, cin))
    for ky in range(3):
        for kx in range(3):
            lxp[ky:ky + H, kx:kx + Wd, :] += lcols[:, :, ky, kx, :]
    # replication padding: padded index q reads x[clamp(q - 1)]
    lx = np.zeros_like(x)
    ry = np.clip(np.arange(H + 2) - 1, 0, H - 1)
    rx = np.clip(np.arange(Wd + 2) - 1, 0, Wd - 1)
    for qy in range(H + 2):
        np.add.at(lx[ry[qy]], rx, lxp[qy])
    return lx, dW, db


def forward(P: G.Plan, u, v, dx, params, S, C, K, omega=1.0, scale=1.0, bf16=False):
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, dx)
    phi0, s, cache = CN.cnn_phi0(P, d, dx, params, S, C, bf16=bf16, keep=True)
    kinv = np.where(P.fluid, 1.0 / np.maximum(P.k, 1.0), 0.0)
    phi = phi0
    for _ in range(K):
        phi = phi - omega * dx * dx * kinv * G.residual(P, d, phi, dx)
    r = G.residual(P, d, phi, dx)
    loss = scale * float(np.sum(r[P.fluid] ** 2))
    return loss, dict(d=d, s=s, cache=cache, phi=phi, r=r, kinv=kinv)


def loss_and_grad(flags, u, v, dx, params, S, C, K, omega=1.0, scale=1.0, bf16=False):
    """Returns (loss, dL/du, dL/dv, dL/dparams) in FP64.

    ``bf16``: the network's forward rounds at the BF16 storage points (as
    cnn.cnn_phi0), and the reverse pass treats every rounding as the
    identity (the straight-through reading of the derivative of a rounding,
    which is zero almost everywhere): it runs at the rounded activations
    with the unrounded weights."""
    P = G.plan(flags)
    loss, F = forward(P, u, v, dx, params, S, C, K, omega, scale, bf16=bf16)
    d, s, cache, r, kinv = F["d"], F["s"], F["cache"], F["r"], F["kinv"]
    nets = CN.unpack(params, S, C)
    fl = P.fluid
    lam_r = np.where(fl, 2.0 * scale * r, 0.0)
    lam_d = lam_r.copy()
    lam = -G.laplacian(P, lam_r, dx)
    for _ in range(K):
        mu = kinv * lam
        lam_d = lam_d - omega * dx * dx * mu
        lam = lam + omega * dx * dx * G.laplacian(P, mu, dx)
    lam_phi0 = np.where(fl, lam, 0.0)
    grads = []
    lam_s = 0.0
    if s > 0.0:
        t0 = cache["t"]
        lam_s += dx * dx * float(np.sum(lam_phi0 * t0))
        lam_t = dx * dx * s * lam_phi0
        lam_y = [None] * S
        for k in range(S - 1):
            lam_y[k] = lam_t
            lam_t = up2_T(lam_t)
        lam_y[S - 1] = lam_t
        lam_x_full = np.zeros(P.shape)
        for k in range(S):
            acts = cache["acts"][k]
            ly = lam_y[k]
            h4 = acts[4]
            dwo = np.einsum("yx,yxc->c", ly, h4)
            dbo = float(ly.sum())
            lam_h = ly[:, :, None] * nets[k]["wo"][None, None, :]
            layer_grads = [None] * 4
            for l in range(3, -1, -1):
                W, b = nets[k]["layers"][l]
                lam_pre = lam_h * (acts[l + 1] > 0)
                lam_h, dW, db = conv3x3_backward(acts[l], W, lam_pre, need_input=True)
                layer_grads[l] = (dW, db)
            lx = lam_h[:, :, 0]
            for _ in range(k):
                lx = down2_T(lx)
            lam_x_full += lx
            for l in range(4):
                grads.append(layer_grads[l][0].ravel())
                grads.append(layer_grads[l][1])
            grads.append(dwo)
            grads.append(np.array([dbo]))
        lam_x_full = np.where(fl, lam_x_full, 0.0)
        lam_d = lam_d + lam_x_full / s
        lam_s -= float(np.sum(lam_x_full * d)) / (s * s)
        lam_d = lam_d + np.where(fl, lam_s * d / (P.nF * s), 0.0)
        dparams = np.concatenate(grads)
    else:
        dparams = np.zeros(CN.param_count(S, C))
    lam_d = np.where(fl, lam_d, 0.0)
    # D^T on open interior faces, open top faces and inflow faces
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


def hybrid_corrected(P: G.Plan, u, v, dx, params, S, C, K, omega=1.0):
    """u - grad(phi) after the CNN guess and K Jacobi sweeps (Eq. 2)."""
    _, F = forward(P, u, v, dx, params, S, C, K, omega)
    ub, vb = G.enforce_bc(P, u, v)
    return G.correct(P, ub, vb, F["phi"], dx)


def long_term(flags, rho, u, v, dx, params, S, C, K, n, alpha, beta, g, rho0, drho, u_in,
              xis, omega=1.0, cfl=0.5):
    """The short-term plus long-term physics-driven loss (Sec. 3.2, Fig. 5,
    Eq. 4) and its gradient with respect to the network parameters.

    Short term: the divergence left after the network's correction of the
    sample u*_t.  Long term: that corrected velocity is advanced n time steps
    (advection and forces, then the same CNN + K sweeps projection) and the
    divergence left after the correction of u*_{t+n} is taken.  Advection is
    not differentiated and the network is frozen inside the unrolled steps,
    so the long-term gradient is the gradient of the last projection's loss
    at the state the rollout reached.  Each term is the sum of squared
    residuals over fluid cells divided by the sum of squared divergences of
    its own input state, weighted by alpha and beta.  xis[j] is the inflow
    perturbation of unrolled step j (j = 0 .. n-1); dt follows the CFL rule.

    Returns dict(loss, loss_short, loss_long, dparams, u_star, v_star, rho).
    """
    assert n >= 1
    P = G.plan(flags)

    def norm(uu, vv):
        d = G.divergence(P, *G.enforce_bc(P, uu, vv), dx)
        return 1.0 / float(np.sum(d[P.fluid] ** 2))

    ls, _, _, gs = loss_and_grad(flags, u, v, dx, params, S, C, K, omega, alpha * norm(u, v))
    uc, vc = hybrid_corrected(P, u, v, dx, params, S, C, K, omega)
    r = np.asarray(rho, np.float64)
    for j in range(n):
        dt = AD.cfl_dt(uc, vc, dx, u_in, cfl)
        r, us, vs = AD.advect_step(P, flags, r, uc, vc, dx, dt, g, rho0, drho, u_in, xis[j])
        if j < n - 1:
            uc, vc = hybrid_corrected(P, us, vs, dx, params, S, C, K, omega)
    ll, _, _, gl = loss_and_grad(flags, us, vs, dx, params, S, C, K, omega, beta * norm(us, vs))
    return dict(loss=ls + ll, loss_short=ls, loss_long=ll, dparams=gs + gl, u_star=us, v_star=vs,
                rho=r)
