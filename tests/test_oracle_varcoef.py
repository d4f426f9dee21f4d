"""Pins of the oracle's variable-density projection (Eq. 2-3 with the cell
density inside the divergence): reduction to the constant-coefficient
operators, the discrete identity div(u - beta grad phi) = d - L_beta phi,
symmetry and definiteness of the face-by-face assembled matrix, a
divergence-free exact solve, the closed form of a horizontally layered
problem, density scaling, and the solvers' convergence to the exact solve."""
import numpy as np
import pytest

import scenes
from oracle import grid as G
from oracle import varcoef as VC


def random_mask_case(n, seed, p_solid=0.2):
    rng = np.random.default_rng(seed)
    flags = np.where(rng.random((n, n)) < p_solid, G.FLAG_SOLID, 0).astype(np.uint8)
    flags[-1, :] = 0  # keep the top row open
    P = G.plan(flags)
    rho = rng.uniform(0.5, 1.0, (n, n))
    return flags, P, rho, rng


def test_constant_density_is_the_constant_operator():
    sc = scenes.plume_scene(24, seed=1, n_obstacles=2)
    P = G.plan(sc.flags)
    bu, bv = VC.face_coefficients(P, np.full(P.shape, 1.3), 1.3)
    rng = np.random.default_rng(0)
    phi = np.where(P.fluid, rng.standard_normal(P.shape), 0.0)
    assert np.allclose(VC.laplacian(P, phi, bu, bv, sc.dx), G.laplacian(P, phi, sc.dx), rtol=1e-13, atol=1e-9)
    assert np.array_equal(VC.diagonal(P, bu, bv), P.k)
    u, v = G.enforce_bc(P, *scenes.random_faces(24, 24, 0, kind="mixed"))
    for a, b in zip(VC.correct(P, u, v, phi, bu, bv, sc.dx), G.correct(P, u, v, phi, sc.dx)):
        assert np.allclose(a, b, rtol=1e-14, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_corrected_divergence_identity(seed):
    sc = scenes.plume_scene(32, seed=seed, n_obstacles=2)
    P = G.plan(sc.flags)
    rho = scenes.random_density(32, 32, seed, 1.0, 0.5)
    bu, bv = VC.face_coefficients(P, rho, 1.0)
    u, v = G.enforce_bc(P, *scenes.random_faces(32, 32, seed, kind="mixed"))
    d = G.divergence(P, u, v, sc.dx)
    phi = np.where(P.fluid, np.random.default_rng(seed).standard_normal(P.shape), 0.0)
    u2, v2 = VC.correct(P, u, v, phi, bu, bv, sc.dx)
    lhs = G.divergence(P, u2, v2, sc.dx)
    rhs = VC.residual(P, d, phi, bu, bv, sc.dx)
    assert np.allclose(lhs, rhs, rtol=1e-12, atol=1e-9 * np.abs(rhs).max())
    # inflow faces are never corrected
    assert np.array_equal(v2[0], v[0])


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_assembled_matrix_symmetric_positive_definite(seed):
    flags, P, rho, rng = random_mask_case(8, seed)
    bu, bv = VC.face_coefficients(P, rho, 1.0)
    A, idx = VC.assemble(P, bu, bv)
    assert np.allclose(A, A.T, rtol=0, atol=1e-14)
    assert np.linalg.eigvalsh(A).min() > 0.0
    # the assembled matrix is the operator: A x = -dx^2 L_beta x
    x = np.where(P.fluid, rng.standard_normal(P.shape), 0.0)
    dx = 1.0 / 8
    assert np.allclose(A @ x[P.fluid], (-(dx * dx) * VC.laplacian(P, x, bu, bv, dx))[P.fluid],
                       rtol=1e-12, atol=1e-12)


def test_exact_solve_is_divergence_free_and_scales_with_density():
    sc = scenes.plume_scene(16, seed=2, n_obstacles=1)
    P = G.plan(sc.flags)
    rho = scenes.random_density(16, 16, 2, 1.0, 0.5)
    bu, bv = VC.face_coefficients(P, rho, 1.0)
    u, v = G.enforce_bc(P, *scenes.random_faces(16, 16, 2, kind="mixed"))
    d = G.divergence(P, u, v, sc.dx)
    phi = VC.exact_solve(P, d, bu, bv, sc.dx)
    u2, v2 = VC.correct(P, u, v, phi, bu, bv, sc.dx)
    assert np.abs(G.divergence(P, u2, v2, sc.dx)).max() < 1e-9 * np.abs(d).max()
    # rho -> c rho divides beta by c, so phi scales by c and the velocity is unchanged
    bu3, bv3 = VC.face_coefficients(P, 3.0 * rho, 1.0)
    phi3 = VC.exact_solve(P, d, bu3, bv3, sc.dx)
    assert np.allclose(phi3, 3.0 * phi, rtol=1e-10, atol=1e-14)


def test_layered_closed_form():
    # all fluid, no inflow, density and vertical velocity varying with height
    # only: fluxes F_{j+1/2} = dx sum_{i<=j} d_i from the bottom wall, then
    # phi from the open top downwards (phi = 0 above the top row).
    n = 12
    P = G.plan(np.zeros((n, n), dtype=np.uint8))
    dx = 1.0 / n
    rng = np.random.default_rng(7)
    rho_y = rng.uniform(0.5, 1.0, n)
    rho = np.repeat(rho_y[:, None], n, axis=1)
    vy = np.concatenate([[0.0], rng.standard_normal(n)])
    u = np.zeros((n, n + 1))
    v = np.repeat(vy[:, None], n, axis=1)
    d = G.divergence(P, u, v, dx)
    bu, bv = VC.face_coefficients(P, rho, 1.0)
    phi = VC.exact_solve(P, d, bu, bv, dx)
    dy = d[:, 0]
    F = dx * np.cumsum(dy)                      # F_{j+1/2}, j = 0..n-1
    beta_face = np.concatenate([1.0 / (0.5 * (rho_y[:-1] + rho_y[1:])), [1.0 / rho_y[-1]]])
    ref = np.zeros(n)
    nxt = 0.0                                   # ghost phi above the top row
    for j in range(n - 1, -1, -1):
        ref[j] = nxt - F[j] * dx / beta_face[j]
        nxt = ref[j]
    assert np.allclose(phi, np.repeat(ref[:, None], n, axis=1), rtol=1e-10, atol=1e-12)


def test_solvers_reach_the_exact_solution():
    flags, P, rho, rng = random_mask_case(12, 9, p_solid=0.15)
    bu, bv = VC.face_coefficients(P, rho, 1.0)
    dx = 1.0 / 12
    u, v = G.enforce_bc(P, rng.standard_normal((12, 13)), rng.standard_normal((13, 12)))
    d = G.divergence(P, u, v, dx)
    ex = VC.exact_solve(P, d, bu, bv, dx)
    phi_j = VC.jacobi(P, d, bu, bv, dx, fixed_iters=20000)[0]
    assert np.allclose(phi_j, ex, rtol=1e-8, atol=1e-10 * np.abs(ex).max())
    phi_c, k, st = VC.pcg(P, d, bu, bv, dx, thr=1e-12 * G.e1(P, d))
    assert st == VC.STATUS_OK and k < 4 * P.nF
    assert np.allclose(phi_c, ex, rtol=1e-7, atol=1e-9 * np.abs(ex).max())
