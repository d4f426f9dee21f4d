"""Pins of the oracle's iterative solvers (Jacobi of Sec. 2.2, PCG baseline)
and of the hybrid stop rule (Sec. 3.3, E_1 of Sec. 4.1)."""
import numpy as np
import pytest

from oracle import grid as G
from oracle import solve as SV
import scenes


def small_problem(seed, n=8, p=0.2):
    rng = np.random.default_rng(seed)
    flags = (rng.random((n, n)) < p).astype(np.uint8)
    P = G.plan(flags)
    d = np.where(P.fluid, rng.standard_normal((n, n)), 0.0)
    return P, d, 1.0 / n, rng


def dense_A(P, dx):
    A, idx = G.assemble(P)
    return A.toarray()


@pytest.mark.parametrize("seed,omega,k", [(0, 1.0, 7), (1, 0.8, 13), (2, 0.6, 1), (3, 1.0, 25)])
def test_jacobi_equals_matrix_power(seed, omega, k):
    # phi_k = M^k phi_0 + sum_{i<k} M^i c with M = I - omega D^-1 A, c = omega D^-1 b
    P, d, dx, rng = small_problem(seed)
    A = dense_A(P, dx)
    Dinv = np.diag(1.0 / np.diag(A))
    b = -(dx * dx) * d[P.fluid]
    x0 = rng.standard_normal(P.nF) * 1e-2
    M = np.eye(P.nF) - omega * Dinv @ A
    c = omega * Dinv @ b
    ref = np.linalg.matrix_power(M, k) @ x0 + sum(np.linalg.matrix_power(M, i) @ c for i in range(k))
    phi0 = np.zeros(P.shape); phi0[P.fluid] = x0
    phi, iters, st, _ = SV.jacobi(P, d, dx, phi0, fixed_iters=k, omega=omega)
    assert iters == k
    assert np.allclose(phi[P.fluid], ref, atol=1e-12 * max(1, np.abs(ref).max()))


def test_jacobi_undamped_is_classic_formula():
    # omega = 1: X_{t+1} = D^-1 (b - (L+U) X_t), the paper's form
    P, d, dx, rng = small_problem(7)
    A = dense_A(P, dx)
    D = np.diag(np.diag(A))
    LU = A - D
    b = -(dx * dx) * d[P.fluid]
    x = np.zeros(P.nF)
    for _ in range(5):
        x = np.linalg.solve(D, b - LU @ x)
    phi, _, _, _ = SV.jacobi(P, d, dx, None, fixed_iters=5)
    assert np.allclose(phi[P.fluid], x, atol=1e-13 * np.abs(x).max())


def test_jacobi_fixed_point_is_exact_solution():
    P, d, dx, _ = small_problem(4, n=6)
    ex = SV.exact_solve(P, d, dx)
    phi, k, st, E = SV.jacobi(P, d, dx, None, thr=1e-11, omega=0.8, max_iters=200000)
    assert st == SV.STATUS_OK
    assert np.abs(phi - ex).max() < 1e-9 * np.abs(ex).max() + 1e-13


def test_jacobi_spectrum_symmetric_on_open_box():
    # the grid graph is bipartite: the spectrum of D^-1 (D - A) is symmetric
    n = 10
    P = G.plan(np.zeros((n, n), dtype=np.uint8))
    A = dense_A(P, 1.0 / n)
    D = np.diag(A)
    Dm = np.diag(D ** -0.5)
    S = np.eye(P.nF) - Dm @ A @ Dm  # similar to D^-1 (D - A)
    ev = np.sort(np.linalg.eigvalsh(S))
    assert np.allclose(ev, -ev[::-1], atol=1e-12)
    assert ev.max() < 1


@pytest.mark.parametrize("seed", range(4))
def test_pcg_finite_termination(seed):
    P, d, dx, _ = small_problem(10 + seed)
    ex = SV.exact_solve(P, d, dx)
    phi, k, st, E = SV.pcg(P, d, dx, None, fixed_iters=P.nF)
    assert np.abs(phi - ex).max() <= 1e-10 * np.abs(ex).max()


def test_pcg_converges_to_threshold_on_plume():
    sc = scenes.plume_scene(32, seed=3, n_obstacles=2)
    u, v = scenes.random_faces(32, 32, 3)
    P = G.plan(sc.flags)
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, sc.dx)
    phi, k, st, E = SV.pcg(P, d, sc.dx, None, thr=1e-6)
    assert st == SV.STATUS_OK and E < 1e-6
    assert E == pytest.approx(G.e1(P, G.residual(P, d, phi, sc.dx)), rel=1e-6)
    assert k < P.nF


def test_stop_rule_check_every_and_maxiter():
    P, d, dx, _ = small_problem(21, n=12)
    e0 = G.e1(P, d)
    # threshold above the initial error: zero sweeps
    phi, k, st, E = SV.jacobi(P, d, dx, None, thr=e0 * 1.0001)
    assert k == 0 and st == SV.STATUS_OK and np.all(phi == 0)
    # strict '<': a threshold equal to E_1 does not stop
    phi, k, st, E = SV.jacobi(P, d, dx, None, thr=e0, max_iters=3)
    assert k >= 1 and E < e0
    phi, k, st, E = SV.jacobi(P, d, dx, None, thr=0.0, max_iters=3)
    assert k == 3 and st == SV.STATUS_MAXITER
    # checks only at multiples of check_every (and at max_iters)
    _, k1, _, _ = SV.jacobi(P, d, dx, None, thr=0.5 * e0, check_every=1)
    _, k5, _, _ = SV.jacobi(P, d, dx, None, thr=0.5 * e0, check_every=5)
    assert k5 % 5 == 0 and k1 <= k5 < k1 + 5
    _, k7, st7, _ = SV.jacobi(P, d, dx, None, thr=0.0, check_every=5, max_iters=7)
    assert k7 == 7 and st7 == SV.STATUS_MAXITER
    # non-finite input
    d2 = d.copy(); d2[P.fluid.nonzero()[0][0], P.fluid.nonzero()[1][0]] = np.nan
    _, k, st, _ = SV.jacobi(P, d2, dx, None, thr=1e-3)
    assert st == SV.STATUS_NONFINITE and k == 0


def test_einf_criterion_stops_on_the_max_residual():
    # E_inf = max |r| (Sec. 4.1's comparison criterion): the returned iterate
    # is the first tested one whose max |r| is below the threshold, so it is
    # later than the E_1 stop at the same threshold (mean <= max), and the
    # tested iterate before it is above the threshold
    import scenes
    sc = scenes.plume_scene(24, seed=3, n_obstacles=1)
    P = G.plan(sc.flags)
    u, v = scenes.random_faces(24, 24, 3, kind="mixed")
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    thr = 0.05 * G.einf(P, d)
    phi, k, st, E = SV.jacobi(P, d, sc.dx, thr=thr, check_every=3, criterion="einf")
    assert st == SV.STATUS_OK and E < thr and k % 3 == 0
    assert G.einf(P, G.residual(P, d, phi, sc.dx)) == E
    prev = SV.jacobi(P, d, sc.dx, fixed_iters=k - 3)[0]
    assert G.einf(P, G.residual(P, d, prev, sc.dx)) >= thr
    k1 = SV.jacobi(P, d, sc.dx, thr=thr, check_every=3)[1]
    assert k1 <= k
    phi_c, kc, stc, Ec = SV.pcg(P, d, sc.dx, thr=thr, criterion="einf")
    assert stc == SV.STATUS_OK and Ec < thr
    assert G.einf(P, G.residual(P, d, phi_c, sc.dx)) < thr
