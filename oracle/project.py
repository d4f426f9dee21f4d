"""Oracle: the full pressure projection of one time step.  Plain FP64.
TEST INFRASTRUCTURE ONLY.

Order of operations (Sec. 2.2 projection step and the hybrid strategy of
Sec. 3.3): plan the flags; enforce the boundary faces; divergence of u*;
initial guess (CNN for the hybrid, zero for the baselines, or a given warm
start); iterate (Jacobi or PCG) until the mean |div| over fluid cells drops
below the threshold; subtract grad phi (Eq. 2); p = rho0 phi / dt.
"""
from __future__ import annotations

import numpy as np

from . import grid as G
from . import solve as SV
from .cnn import cnn_phi0

METHODS = ("hybrid", "jacobi", "pcg", "cnn")


def project(flags, u, v, dx: float, dt: float = 1.0, rho0: float = 1.0,
            threshold: float = 1e-3, method: str = "hybrid", params=None,
            S: int = 3, C: int = 32, bf16: bool = False, omega: float = 1.0,
            check_every: int = 1, max_iters: int = 200000, fixed_iters: int = 0,
            phi_init=None, criterion: str = "e1"):
    assert method in METHODS
    P = G.plan(flags)
    u, v = G.enforce_bc(P, np.asarray(u, np.float64), np.asarray(v, np.float64))
    d = G.divergence(P, u, v, dx)
    e1_init = G.e1(P, d)
    s = 0.0
    if method in ("hybrid", "cnn"):
        phi0, s, _ = cnn_phi0(P, d, dx, params, S, C, bf16=bf16)
    elif phi_init is not None:
        phi0 = np.where(P.fluid, phi_init, 0.0)
    else:
        phi0 = np.zeros(P.shape)
    e1_cnn = G.e1(P, G.residual(P, d, phi0, dx))
    status = SV.STATUS_OK
    if method in ("hybrid", "jacobi"):
        phi, iters, status, _ = SV.jacobi(P, d, dx, phi0, threshold, omega,
                                          check_every, max_iters, fixed_iters, criterion)
    elif method == "pcg":
        phi, iters, status, _ = SV.pcg(P, d, dx, phi0, threshold, check_every,
                                       max_iters, fixed_iters, criterion)
    else:
        phi, iters = phi0, 0
    u2, v2 = G.correct(P, u, v, phi, dx)
    d2 = G.divergence(P, u2, v2, dx)
    return dict(phi=phi, p=rho0 * phi / dt, u=u2, v=v2, iters=iters, status=status,
                e1_init=e1_init, e1_cnn=e1_cnn, e1_final=G.e1(P, d2),
                einf_final=G.einf(P, d2), s=s, plan=P, d=d)
