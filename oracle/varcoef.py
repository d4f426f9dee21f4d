"""Oracle: the variable-density projection, Eq. (3) with the density kept
inside the divergence, div((dt/rho) grad p) = div u*, and Eq. (2) as
u = u* - (dt/rho_f) grad p.  Plain FP64 numpy.  TEST INFRASTRUCTURE ONLY.

The paper writes both equations with the reference density rho0 (its
Boussinesq set-up, Sec. 2.2); this is the variant that keeps the cell
density.  With phi = (dt/rho0) p as elsewhere in this package and the face
coefficient beta_f = rho0 / rho_f,

    (L_beta phi)_c = sum over the open faces f of c of beta_f (phi_nb - phi_c) / dx^2,
    u_f -= beta_f (phi_R - phi_L) / dx   on open faces,

so div(u* - beta grad phi) = d - L_beta phi exactly.  rho_f is the mean of
the two cells' densities on a face between two non-solid cells and the top
cell's density on an open top face (ghost phi = 0); closed faces (walls,
solids) have beta = 0, inflow faces are never corrected.  rho0 = rho
everywhere gives back the constant-coefficient operators of ``grid``.
"""
from __future__ import annotations

import math

import numpy as np

from . import grid as G

STATUS_OK, STATUS_MAXITER, STATUS_NONFINITE = 0, 1, 2


def face_coefficients(P: G.Plan, rho: np.ndarray, rho0: float):
    """(bu (ny, nx+1), bv (ny+1, nx)): beta on every open face, 0 elsewhere."""
    ny, nx = P.shape
    rho = np.asarray(rho, np.float64)
    bu = np.zeros((ny, nx + 1))
    bu[:, 1:nx] = rho0 / (0.5 * (rho[:, :-1] + rho[:, 1:]))
    bv = np.zeros((ny + 1, nx))
    bv[1:ny, :] = rho0 / (0.5 * (rho[:-1, :] + rho[1:, :]))
    bv[ny, :] = rho0 / rho[ny - 1, :]
    return np.where(P.uopen, bu, 0.0), np.where(P.vopen, bv, 0.0)


def laplacian(P: G.Plan, phi: np.ndarray, bu, bv, dx: float) -> np.ndarray:
    """L_beta phi on fluid cells (0 on solids), ghost phi = 0 above the top."""
    ny, nx = P.shape
    z = np.zeros((ny + 1, nx))
    z[:ny] = phi
    fx = bu[:, 1:nx] * (phi[:, 1:] - phi[:, :-1])      # flux through interior u-faces
    fy = bv[1:, :] * (z[1:] - z[:-1])                   # through v-faces 1..ny (top: ghost 0)
    s = np.zeros((ny, nx))
    s[:, :-1] += fx
    s[:, 1:] -= fx
    s += fy
    s[1:, :] -= fy[:-1]
    return np.where(P.fluid, s / (dx * dx), 0.0)


def diagonal(P: G.Plan, bu, bv) -> np.ndarray:
    """Sum of beta over the open faces of each cell (the negated, dx^2-scaled
    diagonal of L_beta)."""
    D = bu[:, 1:] + bu[:, :-1] + bv[1:, :] + bv[:-1, :]
    return np.where(P.fluid, D, 0.0)


def residual(P, d, phi, bu, bv, dx):
    return np.where(P.fluid, d - laplacian(P, phi, bu, bv, dx), 0.0)


def correct(P: G.Plan, u, v, phi, bu, bv, dx: float):
    """u -= beta grad phi on the open faces (inflow and closed faces keep
    their values)."""
    ny, nx = P.shape
    u = u.copy()
    v = v.copy()
    u[:, 1:nx] -= bu[:, 1:nx] * (phi[:, 1:] - phi[:, :-1]) / dx
    v[1:ny, :] -= bv[1:ny, :] * (phi[1:, :] - phi[:-1, :]) / dx
    v[ny, :] -= bv[ny, :] * (0.0 - phi[ny - 1, :]) / dx
    return u, v


def assemble(P: G.Plan, bu, bv):
    """A = -dx^2 L_beta on the fluid cells as a dense matrix (small grids),
    built face by face, with the fluid-cell index map."""
    ny, nx = P.shape
    idx = -np.ones((ny, nx), dtype=np.int64)
    idx[P.fluid] = np.arange(P.nF)
    A = np.zeros((P.nF, P.nF))
    for j in range(ny):
        for i in range(nx):
            if not P.fluid[j, i]:
                continue
            c = idx[j, i]
            for (b, jj, ii) in ((bu[j, i + 1], j, i + 1), (bu[j, i], j, i - 1),
                                (bv[j + 1, i], j + 1, i), (bv[j, i], j - 1, i)):
                if b == 0.0:
                    continue
                A[c, c] += b
                if 0 <= jj < ny and 0 <= ii < nx:  # the ghost row has no unknown
                    A[c, idx[jj, ii]] -= b
    return A, idx


def exact_solve(P: G.Plan, d, bu, bv, dx: float) -> np.ndarray:
    A, idx = assemble(P, bu, bv)
    x = np.linalg.solve(A, -(dx * dx) * d[P.fluid])
    phi = np.zeros(P.shape)
    phi[P.fluid] = x
    return phi


def _test_due(k, check_every, max_iters):
    return k % check_every == 0 or k >= max_iters


def jacobi(P, d, bu, bv, dx, phi0=None, thr=0.0, omega=1.0, check_every=1, max_iters=200000,
           fixed_iters=0):
    """Weighted Jacobi phi <- phi - omega dx^2 r / D; the stop rule of the
    constant-coefficient solver.  Returns (phi, iters, status)."""
    phi = np.zeros(P.shape) if phi0 is None else np.where(P.fluid, phi0, 0.0)
    D = diagonal(P, bu, bv)
    Dinv = np.where(P.fluid, 1.0 / np.where(D > 0, D, 1.0), 0.0)
    k = 0
    while True:
        r = residual(P, d, phi, bu, bv, dx)
        if fixed_iters > 0:
            if k >= fixed_iters:
                return phi, k, STATUS_OK
        elif _test_due(k, check_every, max_iters):
            E = G.e1(P, r)
            if not math.isfinite(E):
                return phi, k, STATUS_NONFINITE
            if E < thr:
                return phi, k, STATUS_OK
            if k >= max_iters:
                return phi, k, STATUS_MAXITER
        phi = phi - omega * dx * dx * Dinv * r
        k += 1


def pcg(P, d, bu, bv, dx, thr=0.0, check_every=1, max_iters=100000):
    """Diagonally preconditioned CG on A x = -dx^2 d.  Returns (phi, iters, status)."""
    A = lambda x: -(dx * dx) * laplacian(P, x, bu, bv, dx)
    D = diagonal(P, bu, bv)
    Dinv = np.where(P.fluid, 1.0 / np.where(D > 0, D, 1.0), 0.0)
    x = np.zeros(P.shape)
    r = np.where(P.fluid, -(dx * dx) * d, 0.0)
    z = r * Dinv
    p = z.copy()
    rz = float(np.sum(r * z))
    k = 0
    while True:
        if _test_due(k, check_every, max_iters):
            E = G.e1(P, r) / (dx * dx)
            if E < thr:
                return x, k, STATUS_OK
            if k >= max_iters:
                return x, k, STATUS_MAXITER
        q = A(p)
        pq = float(np.sum(p * q))
        if pq <= 0.0:
            return x, k, STATUS_OK
        a = rz / pq
        x = x + a * p
        r = r - a * q
        z = r * Dinv
        rz_new = float(np.sum(r * z))
        p = z + (rz_new / rz) * p
        rz = rz_new
        k += 1
