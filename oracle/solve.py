"""Oracle: Poisson solvers for L phi = d (Eq. 3).  Plain FP64.
TEST INFRASTRUCTURE ONLY.

* ``exact_solve``: direct solve of A phi = b with A = -dx^2 L and b = -dx^2 d
  (dense LAPACK for small systems, sparse direct otherwise); the paper's
  "direct method" of Sec. 2.2 used as ground truth.
* ``jacobi``: X_{t+1} = D^-1 (b - (L+U) X_t) of Sec. 2.2, written in the
  equivalent correction form phi <- phi - omega dx^2 r / k_c with the
  residual r = d - L phi; omega = 1 is the paper's undamped iteration.
* ``pcg``: textbook conjugate gradient on A phi = b with the Jacobi
  preconditioner M = diag(k_c) (the Krylov baseline).

Stop rule shared by the iterative solvers (the hybrid criterion of
Sec. 3.3 / Sec. 4.1): the mean |r| over fluid cells of the current iterate
is tested before the first update (k = 0), after every ``check_every``
updates and at ``k = max_iters``; the first tested iterate with E_1 < thr
(strict) is returned.  ``criterion="einf"`` tests E_inf = max |r| over fluid
cells instead (the criterion of the prior hybrid work that Sec. 4.1
compares against).  ``fixed_iters > 0`` ignores the threshold and returns
the iterate after exactly that many updates.
"""
from __future__ import annotations

import math

import numpy as np

from . import grid as G

STATUS_OK = 0
STATUS_MAXITER = 1
STATUS_NONFINITE = 2


def exact_solve(P: G.Plan, d: np.ndarray, dx: float) -> np.ndarray:
    A, idx = G.assemble(P)
    b = -(dx * dx) * d[P.fluid]
    if P.nF == 0:
        return np.zeros(P.shape)
    if P.nF <= 4096:
        x = np.linalg.solve(A.toarray(), b)
    else:
        from scipy.sparse.linalg import spsolve
        x = spsolve(A.tocsc(), b)
    phi = np.zeros(P.shape)
    phi[P.fluid] = x
    return phi


def _test_due(k, check_every, max_iters):
    return (k % check_every == 0) or (k == max_iters)


def _measure(criterion):
    return G.einf if criterion == "einf" else G.e1


def jacobi(P: G.Plan, d: np.ndarray, dx: float, phi0=None, thr: float = 0.0,
           omega: float = 1.0, check_every: int = 1, max_iters: int = 200000,
           fixed_iters: int = 0, criterion: str = "e1"):
    """Returns (phi, iters, status, measure_of_returned_iterate)."""
    measure = _measure(criterion)
    phi = np.zeros(P.shape) if phi0 is None else np.where(P.fluid, phi0, 0.0)
    kinv = np.where(P.fluid, 1.0 / np.maximum(P.k, 1.0), 0.0)
    k = 0
    while True:
        r = G.residual(P, d, phi, dx)
        if fixed_iters > 0:
            if k >= fixed_iters:
                return phi, k, STATUS_OK, measure(P, r)
        elif _test_due(k, check_every, max_iters):
            E = measure(P, r)
            if not math.isfinite(E):
                return phi, k, STATUS_NONFINITE, E
            if E < thr:
                return phi, k, STATUS_OK, E
            if k >= max_iters:
                return phi, k, STATUS_MAXITER, E
        phi = phi - omega * dx * dx * r * kinv
        k += 1


def apply_A(P: G.Plan, x: np.ndarray, dx: float) -> np.ndarray:
    """A x = -dx^2 L x (symmetric positive definite on fluid cells)."""
    return -(dx * dx) * G.laplacian(P, x, dx)


def pcg(P: G.Plan, d: np.ndarray, dx: float, phi0=None, thr: float = 0.0,
        check_every: int = 1, max_iters: int = 100000, fixed_iters: int = 0,
        criterion: str = "e1"):
    """Jacobi-preconditioned CG.  Returns (phi, iters, status, measure)."""
    measure = _measure(criterion)
    x = np.zeros(P.shape) if phi0 is None else np.where(P.fluid, phi0, 0.0)
    b = -(dx * dx) * d
    kinv = np.where(P.fluid, 1.0 / np.maximum(P.k, 1.0), 0.0)
    r = np.where(P.fluid, b - apply_A(P, x, dx), 0.0)
    z = r * kinv
    p = z.copy()
    rz = float(np.sum(r * z))
    k = 0
    inv_dx2 = 1.0 / (dx * dx)
    while True:
        E = measure(P, r) * inv_dx2  # r here is -dx^2 (d - L x)
        if fixed_iters > 0:
            if k >= fixed_iters:
                return x, k, STATUS_OK, E
        elif _test_due(k, check_every, max_iters):
            if not math.isfinite(E):
                return x, k, STATUS_NONFINITE, E
            if E < thr:
                return x, k, STATUS_OK, E
            if k >= max_iters:
                return x, k, STATUS_MAXITER, E
        q = apply_A(P, p, dx)
        pq = float(np.sum(p * q))
        if pq <= 0.0:  # exact convergence (p = 0) or breakdown
            return x, k, STATUS_OK, E
        alpha = rz / pq
        x = x + alpha * p
        r = r - alpha * q
        z = r * kinv
        rz_new = float(np.sum(r * z))
        beta = rz_new / rz if rz != 0.0 else 0.0
        p = z + beta * p
        rz = rz_new
        k += 1
