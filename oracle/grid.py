"""Oracle: MAC grid, flags planner, divergence, masked Laplacian, gradient
correction.  Plain FP64 numpy.  TEST INFRASTRUCTURE ONLY: nothing in the
product path may import this package.

Conventions (MAC staggering of the numerical set-up, paper Sec. 2.2):

* cells (i, j), i = 0..nx-1 (x), j = 0..ny-1 (y, j = 0 at the bottom),
  arrays indexed ``[j, i]``;
* ``u[j, i]``, i = 0..nx: x-face on the left of cell (i, j), shape (ny, nx+1);
* ``v[j, i]``, j = 0..ny: y-face below cell (i, j), shape (ny+1, nx);
* left, right and bottom domain edges are solid walls, the top is open: an
  implicit ghost row j = ny of empty cells with pressure 0;
* bottom faces of cells flagged INFLOW carry a prescribed velocity that the
  projection never changes.

The scaled pressure phi = (dt / rho0) p turns Eq. (3) into L phi = div u*
and Eq. (2) into u = u* - grad phi.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import ndimage

FLAG_SOLID = 1
FLAG_INFLOW = 2


@dataclass
class Plan:
    """Result of the planning step (hot-path row a0)."""
    fluid: np.ndarray   # (ny, nx) bool, after pocket fill
    nE: np.ndarray      # (ny, nx) bool: east neighbour is a non-solid cell
    nW: np.ndarray
    nN: np.ndarray      # north neighbour non-solid, or the open ghost row
    nS: np.ndarray
    k: np.ndarray       # (ny, nx) float64 count of non-solid neighbours (0 on solid)
    uopen: np.ndarray   # (ny, nx+1) bool: face between two non-solid cells
    vopen: np.ndarray   # (ny+1, nx) bool: idem; top row = open boundary faces
    vinflow: np.ndarray  # (nx,) bool: prescribed inflow face below row 0
    nF: int

    @property
    def shape(self):
        return self.fluid.shape


def pocket_fill(solid: np.ndarray) -> np.ndarray:
    """Fluid cells that no 4-connected path of non-solid cells links to the
    open top row become solid (an enclosed pocket makes the Poisson matrix
    singular).  Returns the new solid mask."""
    fluid = ~solid
    lab, n = ndimage.label(fluid, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    top = np.unique(lab[-1][lab[-1] > 0])
    keep = np.isin(lab, top)
    return ~keep


def plan(flags: np.ndarray) -> Plan:
    flags = np.asarray(flags, dtype=np.uint8)
    ny, nx = flags.shape
    solid = pocket_fill((flags & FLAG_SOLID) != 0)
    fluid = ~solid
    nE = np.zeros_like(fluid)
    nW = np.zeros_like(fluid)
    nN = np.zeros_like(fluid)
    nS = np.zeros_like(fluid)
    nE[:, :-1] = fluid[:, 1:]
    nW[:, 1:] = fluid[:, :-1]
    nS[1:, :] = fluid[:-1, :]
    nN[:-1, :] = fluid[1:, :]
    nN[-1, :] = True  # open top: the ghost row is a non-solid neighbour
    nE &= fluid
    nW &= fluid
    nN &= fluid
    nS &= fluid
    k = (nE.astype(np.int64) + nW + nN + nS).astype(np.float64)
    uopen = np.zeros((ny, nx + 1), dtype=bool)
    uopen[:, 1:nx] = fluid[:, :-1] & fluid[:, 1:]
    vopen = np.zeros((ny + 1, nx), dtype=bool)
    vopen[1:ny, :] = fluid[:-1, :] & fluid[1:, :]
    vopen[ny, :] = fluid[ny - 1, :]
    vinflow = fluid[0, :] & ((flags[0, :] & FLAG_INFLOW) != 0)
    return Plan(fluid=fluid, nE=nE, nW=nW, nN=nN, nS=nS, k=k, uopen=uopen,
                vopen=vopen, vinflow=vinflow, nF=int(fluid.sum()))


def enforce_bc(P: Plan, u: np.ndarray, v: np.ndarray):
    """Zero every face that touches a solid cell or a wall; keep inflow faces."""
    u = np.where(P.uopen, u, 0.0)
    v = v.copy()
    v[1:, :] = np.where(P.vopen[1:, :], v[1:, :], 0.0)
    v[0, :] = np.where(P.vinflow, v[0, :], 0.0)
    return u, v


def divergence(P: Plan, u: np.ndarray, v: np.ndarray, dx: float) -> np.ndarray:
    """First-order forward-difference divergence on fluid cells (Sec. 3.2),
    zero on solid cells.  Faces are taken as given (call enforce_bc first)."""
    d = (u[:, 1:] - u[:, :-1] + v[1:, :] - v[:-1, :]) / dx
    return np.where(P.fluid, d, 0.0)


def laplacian(P: Plan, phi: np.ndarray, dx: float) -> np.ndarray:
    """Masked 5-point Laplacian of Eq. (3): sum over non-solid neighbours of
    (phi_n - phi_c) / dx^2, with phi = 0 on the open ghost row; 0 on solid."""
    ny, nx = phi.shape
    z = np.zeros((ny + 2, nx + 2))
    z[1:-1, 1:-1] = phi
    E = z[1:-1, 2:]
    W = z[1:-1, :-2]
    N = z[2:, 1:-1]   # row ny (ghost) stays 0
    S = z[:-2, 1:-1]
    s = P.nE * (E - phi) + P.nW * (W - phi) + P.nN * (N - phi) + P.nS * (S - phi)
    return np.where(P.fluid, s / (dx * dx), 0.0)


def residual(P: Plan, d: np.ndarray, phi: np.ndarray, dx: float) -> np.ndarray:
    """r = d - L phi, which is the divergence of u* - grad phi."""
    return np.where(P.fluid, d - laplacian(P, phi, dx), 0.0)


def correct(P: Plan, u: np.ndarray, v: np.ndarray, phi: np.ndarray, dx: float):
    """Eq. (2): subtract grad phi on every face between two non-solid cells,
    including the open top faces (ghost phi = 0)."""
    u = u.copy()
    v = v.copy()
    u[:, 1:-1] -= P.uopen[:, 1:-1] * (phi[:, 1:] - phi[:, :-1]) / dx
    v[1:-1, :] -= P.vopen[1:-1, :] * (phi[1:, :] - phi[:-1, :]) / dx
    v[-1, :] -= P.vopen[-1, :] * (0.0 - phi[-1, :]) / dx
    return u, v


def e1(P: Plan, r: np.ndarray) -> float:
    """Mean |div u| over fluid cells (the hybrid's stop quantity, Sec. 4.1)."""
    if P.nF == 0:
        return 0.0
    return float(np.abs(r[P.fluid]).sum() / P.nF)


def einf(P: Plan, r: np.ndarray) -> float:
    """Max |div u| over fluid cells."""
    if P.nF == 0:
        return 0.0
    return float(np.abs(r[P.fluid]).max())


def assemble(P: Plan):
    """A = -dx^2 L restricted to fluid cells, as a scipy CSR matrix with the
    fluid-cell index map: diagonal k_c, -1 per non-solid neighbour."""
    from scipy import sparse
    ny, nx = P.shape
    idx = -np.ones((ny, nx), dtype=np.int64)
    idx[P.fluid] = np.arange(P.nF)
    rows, cols, vals = [], [], []
    jj, ii = np.nonzero(P.fluid)
    c = idx[jj, ii]
    rows.append(c); cols.append(c); vals.append(P.k[jj, ii])
    for mask, dj, di in ((P.nE, 0, 1), (P.nW, 0, -1), (P.nS, -1, 0), (P.nN, 1, 0)):
        sel = mask[jj, ii]
        j2 = jj[sel] + dj
        i2 = ii[sel] + di
        inside = j2 < ny  # the ghost row has no unknown
        rows.append(c[sel][inside])
        cols.append(idx[j2[inside], i2[inside]])
        vals.append(-np.ones(int(inside.sum())))
    A = sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(P.nF, P.nF))
    return A, idx
