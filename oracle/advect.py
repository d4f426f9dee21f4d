"""Oracle: the advection/force half of a time step, producing u*.
Plain FP64.  TEST INFRASTRUCTURE ONLY.

Sec. 2.2: density advected as a passive scalar by a MacCormack
semi-Lagrangian scheme (Selle et al. 2008), velocity advected the same way,
then the external (buoyancy) force by forward Euler.

Readings taken where the paper is silent:
* all three fields are advected with the start-of-step velocity, traced
  back with one Euler step, sampled bilinearly with positions clamped to the
  sampled grid's extent;
* MacCormack: q_hat = SL(q, dt), q_tilde = SL(q_hat, -dt),
  q_new = q_hat + (q - q_tilde)/2, then clamped to the min/max of the four
  samples that the forward trace interpolated (the limiter);
* buoyancy on interior and top v-faces: v += dt g (rho0 - rho_f)/rho0 with
  rho_f the mean of the two adjacent cells (top face: the cell below);
* inflow faces get U_in (1 + xi), inflow cells rho0 (1 - drho); then every
  face touching a solid cell or a wall is zeroed;
* dt = cfl dx / max(max|u|, max|v|, U_in) from the state at the step start.
"""
from __future__ import annotations

import numpy as np

from . import grid as G


def _sample(q: np.ndarray, X: np.ndarray, Y: np.ndarray):
    """Bilinear sample of q (indexed [j, i] at integer coords (i, j)) at
    continuous index coords, clamped; returns (value, min4, max4)."""
    H, W = q.shape
    X = np.clip(X, 0.0, W - 1)
    Y = np.clip(Y, 0.0, H - 1)
    i0 = np.minimum(np.floor(X).astype(np.int64), max(W - 2, 0))
    j0 = np.minimum(np.floor(Y).astype(np.int64), max(H - 2, 0))
    fx = X - i0
    fy = Y - j0
    i1 = np.minimum(i0 + 1, W - 1)
    j1 = np.minimum(j0 + 1, H - 1)
    a = q[j0, i0]; b = q[j0, i1]; c = q[j1, i0]; d = q[j1, i1]
    val = (1 - fy) * ((1 - fx) * a + fx * b) + fy * ((1 - fx) * c + fx * d)
    mn = np.minimum(np.minimum(a, b), np.minimum(c, d))
    mx = np.maximum(np.maximum(a, b), np.maximum(c, d))
    return val, mn, mx


def _vel_at_centres(u, v):
    return 0.5 * (u[:, :-1] + u[:, 1:]), 0.5 * (v[:-1, :] + v[1:, :])


def _vel_at_ufaces(u, v):
    ny, nx1 = u.shape
    nx = nx1 - 1
    il = np.clip(np.arange(nx + 1) - 1, 0, nx - 1)
    ir = np.clip(np.arange(nx + 1), 0, nx - 1)
    vv = 0.25 * (v[:-1, il] + v[:-1, ir] + v[1:, il] + v[1:, ir])
    return u, vv


def _vel_at_vfaces(u, v):
    ny1, nx = v.shape
    ny = ny1 - 1
    jb = np.clip(np.arange(ny + 1) - 1, 0, ny - 1)
    jt = np.clip(np.arange(ny + 1), 0, ny - 1)
    uu = 0.25 * (u[jb, :-1] + u[jb, 1:] + u[jt, :-1] + u[jt, 1:])
    return uu, v


def maccormack(q: np.ndarray, velx: np.ndarray, vely: np.ndarray, dt_over_dx: float):
    """Advect q sampled at integer index coords with velocities (in cells per
    unit time x dx) given at the same sample points."""
    H, W = q.shape
    I, J = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    ox = dt_over_dx * velx
    oy = dt_over_dx * vely
    q_hat, mn, mx = _sample(q, I - ox, J - oy)
    q_til, _, _ = _sample(q_hat, I + ox, J + oy)
    q_new = q_hat + 0.5 * (q - q_til)
    return np.clip(q_new, mn, mx)


def cfl_dt(u, v, dx: float, u_in: float, cfl: float = 0.5) -> float:
    m = max(float(np.abs(u).max()), float(np.abs(v).max()), u_in)
    return cfl * dx / m


def advect_step(P: G.Plan, flags, rho, u, v, dx: float, dt: float, g: float,
                rho0: float, drho: float, u_in: float, xi: np.ndarray):
    """One advection + force step.  Returns (rho_new, u_star, v_star)."""
    r = dt / dx
    rho_n = maccormack(rho, *_vel_at_centres(u, v), r)
    u_n = maccormack(u, *_vel_at_ufaces(u, v), r)
    v_n = maccormack(v, *_vel_at_vfaces(u, v), r)
    ny, nx = rho.shape
    rf = np.empty((ny + 1, nx))
    rf[1:ny] = 0.5 * (rho_n[:-1] + rho_n[1:])
    rf[ny] = rho_n[ny - 1]
    v_n[1:] += dt * g * (rho0 - rf[1:]) / rho0
    rho_n[0, P.vinflow] = rho0 * (1.0 - drho)
    v_n[0] = np.where(P.vinflow, u_in * (1.0 + xi), 0.0)
    u_s, v_s = G.enforce_bc(P, u_n, v_n)
    return rho_n, u_s, v_s
