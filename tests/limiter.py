"""Where the MacCormack limiter of the advection may legitimately differ
between the FP32 GPU step and the FP64 oracle (test helpers, CPU only).

The limiter (Sec. 2.2, MacCormack with the min/max clamp of Selle et al.)
bounds the corrected value by the extremes of the four grid samples around
the back-trace point.  Bilinear sampling is continuous in the position, but
the choice of those four samples is not: where the back-trace lands within
rounding of a grid line, FP32 and FP64 may take neighbouring sample cells
and so different bounds.  ``ambiguous`` flags exactly those points (the
back-trace within ``eps`` of an interior grid line in either direction);
everywhere else both sides make the same discrete choice and must agree to
rounding.  At a flagged point either choice is legitimate, so the GPU's
value must match the oracle's correction clamped to the bounds of one of
the sample cells a back-trace within rounding could select
(``limiter_candidates``).
"""
from __future__ import annotations

import numpy as np

from oracle import advect as AD


def trace_positions(u, v, dt: float, dx: float):
    """Back-trace index positions (X, Y), clamped like the sampling, of the
    three sample grids (cell centres, u faces, v faces), with the velocity
    components at the sample points (a zero component leaves the position on
    its grid line exactly, in any precision)."""
    r = dt / dx
    out = []
    for vx, vy in (AD._vel_at_centres(u, v), AD._vel_at_ufaces(u, v), AD._vel_at_vfaces(u, v)):
        H, W = vx.shape
        J, I = np.mgrid[0:H, 0:W].astype(np.float64)
        out.append((np.clip(I - r * vx, 0.0, W - 1.0), np.clip(J - r * vy, 0.0, H - 1.0), vx, vy))
    return out


def position_eps(H: int, W: int) -> float:
    """Rounding allowance of an FP32 back-trace position: eight units in the
    last place of the largest index."""
    return 8.0 * max(H, W) * 2.0 ** -24


def ambiguous(X, Y, H: int, W: int, eps: float, vx=None, vy=None):
    """Back-trace within eps of an interior grid line (at the clamped ends
    the sample cell is pinned and no choice arises; nor does it where the
    velocity component is exactly zero)."""
    def near(P, n, vel):
        f = P - np.floor(P)
        m = (np.minimum(f, 1.0 - f) < eps) & (P > eps) & (P < n - 1 - eps)
        return m if vel is None else m & (vel != 0)
    return near(X, W, vx) | near(Y, H, vy)


def limiter_candidates(q, vx, vy, r: float, eps: float):
    """The results the MacCormack step can legitimately give at every sample
    point of q: the unclamped correction of the oracle, clamped to the
    bounds of each sample cell that a back-trace within eps of the oracle's
    selects (up to four).  Returns (candidates, ambiguous mask)."""
    H, W = q.shape
    J, I = np.mgrid[0:H, 0:W].astype(np.float64)
    ox, oy = r * vx, r * vy
    q_hat = AD._sample(q, I - ox, J - oy)[0]
    q_til = AD._sample(q_hat, I + ox, J + oy)[0]
    q_new = q_hat + 0.5 * (q - q_til)
    X = np.clip(I - ox, 0.0, W - 1.0)
    Y = np.clip(J - oy, 0.0, H - 1.0)
    cands = []
    for sx in (-eps, eps):
        i0 = np.minimum(np.floor(np.clip(X + sx, 0.0, W - 1.0)).astype(np.int64), max(W - 2, 0))
        i1 = np.minimum(i0 + 1, W - 1)
        for sy in (-eps, eps):
            j0 = np.minimum(np.floor(np.clip(Y + sy, 0.0, H - 1.0)).astype(np.int64), max(H - 2, 0))
            j1 = np.minimum(j0 + 1, H - 1)
            c4 = (q[j0, i0], q[j0, i1], q[j1, i0], q[j1, i1])
            cands.append(np.clip(q_new, np.minimum.reduce(c4), np.maximum.reduce(c4)))
    return cands, ambiguous(X, Y, H, W, eps, vx, vy)


def compare_advected(P, rho_in, u_in, v_in, dt, dx, g, rho0, out_gpu, out_oracle, tol):
    """Element-wise comparison of an advection + force step (rho, u*, v*)
    with the oracle's from the same inputs.  Every point agrees with the
    oracle to tol * max|field|, or is flagged ambiguous and agrees as
    closely with one of its limiter candidates (after the same inflow,
    buoyancy and wall handling).  A v face next to an ambiguous density cell
    may also carry the buoyancy of that cell's candidates' spread."""
    ny, nx = rho_in.shape
    r = dt / dx
    eps = position_eps(ny + 1, nx + 1)
    vels = (AD._vel_at_centres(u_in, v_in), AD._vel_at_ufaces(u_in, v_in),
            AD._vel_at_vfaces(u_in, v_in))
    rho_o = out_oracle[0]
    rep = {}
    extra_v = np.zeros((ny + 1, nx))
    for k, name in enumerate(("rho", "u", "v")):
        q = (rho_in, u_in, v_in)[k]
        cands, amb = limiter_candidates(q, vels[k][0], vels[k][1], r, eps)
        if k == 0:
            cands = [c.copy() for c in cands]
            for c in cands:
                c[0, P.vinflow] = rho_o[0, P.vinflow]
            amb[0, P.vinflow] = False
            spread = np.where(amb, np.max(cands, axis=0) - np.min(cands, axis=0), 0.0)
            # a face's density is the mean of its two cells (the top face:
            # the cell below), so the two cells' spreads add
            w = 0.5 * dt * abs(g) * spread / rho0
            extra_v[1:ny] = w[:-1] + w[1:]
            extra_v[ny] = 2.0 * w[ny - 1]
        elif k == 1:
            cands = [np.where(P.uopen, c, 0.0) for c in cands]
        else:
            rf = np.empty((ny + 1, nx))
            rf[1:ny] = 0.5 * (rho_o[:-1] + rho_o[1:])
            rf[ny] = rho_o[ny - 1]
            out = []
            for c in cands:
                c = c.copy()
                c[1:] += dt * g * (rho0 - rf[1:]) / rho0
                c[0] = out_oracle[2][0]
                c[1:] = np.where(P.vopen[1:], c[1:], 0.0)
                out.append(c)
            cands = out
            amb = amb | (extra_v > 0)
            amb[0] = False
            amb[1:] &= P.vopen[1:]
        a, b = out_gpu[k], out_oracle[k]
        scale = max(float(np.abs(b).max()), 1e-30)
        slack = tol * scale + (extra_v if k == 2 else 0.0)
        diff = np.abs(a - b)
        near_cand = np.min([np.abs(a - c) for c in cands], axis=0) <= slack
        clear = diff <= tol * scale
        bad = ~clear & ~(amb & near_cand)
        rep[name] = dict(n=a.size, n_amb=int(amb.sum()), n_bad=int(bad.sum()),
                         n_flipped=int((~clear).sum()),
                         max_rel_clear=float((diff[~amb].max() if (~amb).any() else 0.0) / scale),
                         bad_idx=np.argwhere(bad)[:5].tolist())
    return rep
