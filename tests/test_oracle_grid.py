"""Pins of the oracle's grid operators against closed forms, brute force and
invariants (Eq. 2/3 of Sec. 2.2, the divergence of Sec. 3.2)."""
from collections import deque

import numpy as np
import pytest

from oracle import grid as G
from oracle import solve as SV
from oracle import project as PR
import scenes


def open_box(n, ny=None):
    ny = n if ny is None else ny
    return np.zeros((ny, n), dtype=np.uint8)


def random_mask(rng, nx, ny, p=0.25):
    return (rng.random((ny, nx)) < p).astype(np.uint8)


# ---- closed form: discrete eigenmodes of the walls + open-top Laplacian ----

@pytest.mark.parametrize("N,k,m", [(8, 0, 0), (8, 3, 2), (16, 5, 7), (16, 15, 0), (12, 1, 11)])
def test_eigenmode_mixed_bc(N, k, m):
    # Neumann on left/right/bottom, phi = 0 on the ghost row above the top:
    # phi_ij = cos(pi k (i+1/2)/N) cos(pi (m+1/2)(j+1/2)/(N+1/2)),
    # A phi = lambda phi with lambda = 4 sin^2(pi k/2N) + 4 sin^2(pi (m+1/2)/(2N+1)).
    dx = 1.0 / N
    P = G.plan(open_box(N))
    i = np.arange(N)[None, :]
    j = np.arange(N)[:, None]
    phi = np.cos(np.pi * k * (i + 0.5) / N) * np.cos(np.pi * (m + 0.5) * (j + 0.5) / (N + 0.5))
    lam = 4 * np.sin(np.pi * k / (2 * N)) ** 2 + 4 * np.sin(np.pi * (m + 0.5) / (2 * N + 1)) ** 2
    Aphi = -(dx * dx) * G.laplacian(P, phi, dx)
    assert np.allclose(Aphi, lam * phi, atol=1e-13 * max(1, lam))
    d = -lam * phi / (dx * dx)
    sol = SV.exact_solve(P, d, dx)
    assert np.linalg.norm(sol - phi) <= 1e-11 * np.linalg.norm(phi)


def test_eigenmode_rectangular():
    nx, ny, k, m = 10, 6, 3, 4
    dx = 1.0 / nx
    P = G.plan(open_box(nx, ny))
    i = np.arange(nx)[None, :]
    j = np.arange(ny)[:, None]
    phi = np.cos(np.pi * k * (i + 0.5) / nx) * np.cos(np.pi * (m + 0.5) * (j + 0.5) / (ny + 0.5))
    lam = 4 * np.sin(np.pi * k / (2 * nx)) ** 2 + 4 * np.sin(np.pi * (m + 0.5) / (2 * ny + 1)) ** 2
    assert np.allclose(-(dx * dx) * G.laplacian(P, phi, dx), lam * phi, atol=1e-13)


# ---- brute force: the matrix written cell by cell --------------------------

def brute_matrix(flags):
    """A = -dx^2 L assembled with explicit loops from the definition."""
    ny, nx = flags.shape
    solid = pocket_fill_bfs(flags & 1)
    cells = [(j, i) for j in range(ny) for i in range(nx) if not solid[j][i]]
    index = {c: n for n, c in enumerate(cells)}
    A = np.zeros((len(cells), len(cells)))
    for (j, i), r in index.items():
        for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            jj, ii = j + dj, i + di
            if jj == ny:  # open top: ghost neighbour with phi = 0
                A[r, r] += 1
                continue
            if jj < 0 or ii < 0 or ii >= nx or solid[jj][ii]:
                continue
            A[r, r] += 1
            A[r, index[(jj, ii)]] -= 1
    return A, cells, solid


def pocket_fill_bfs(solid_in):
    ny, nx = solid_in.shape
    solid = [[bool(solid_in[j, i]) for i in range(nx)] for j in range(ny)]
    seen = [[False] * nx for _ in range(ny)]
    q = deque()
    for i in range(nx):
        if not solid[ny - 1][i]:
            seen[ny - 1][i] = True
            q.append((ny - 1, i))
    while q:
        j, i = q.popleft()
        for dj, di in ((0, 1), (0, -1), (1, 0), (-1, 0)):
            jj, ii = j + dj, i + di
            if 0 <= jj < ny and 0 <= ii < nx and not solid[jj][ii] and not seen[jj][ii]:
                seen[jj][ii] = True
                q.append((jj, ii))
    return [[solid[j][i] or not seen[j][i] for i in range(nx)] for j in range(ny)]


@pytest.mark.parametrize("seed", range(6))
def test_pocket_fill_matches_bfs(seed):
    rng = np.random.default_rng(seed)
    flags = random_mask(rng, 11, 9, p=0.35)
    P = G.plan(flags)
    ref = np.array(pocket_fill_bfs(flags & 1))
    assert np.array_equal(~P.fluid, ref)


@pytest.mark.parametrize("seed", range(5))
def test_bruteforce_dense_8x8(seed):
    rng = np.random.default_rng(100 + seed)
    flags = random_mask(rng, 8, 8, p=0.2)
    dx = 1.0 / 8
    A_bf, cells, solid = brute_matrix(flags)
    P = G.plan(flags)
    A, idx = G.assemble(P)
    assert np.array_equal(A.toarray(), A_bf)
    # operator form agrees with the matrix
    x = rng.standard_normal(len(cells))
    phi = np.zeros((8, 8))
    for n, (j, i) in enumerate(cells):
        phi[j, i] = x[n]
    Ax = -(dx * dx) * G.laplacian(P, phi, dx)
    assert np.allclose([Ax[j, i] for (j, i) in cells], A_bf @ x, atol=1e-13)
    # exact solve equals numpy's dense solve of the brute-force matrix
    d = np.where(P.fluid, rng.standard_normal((8, 8)), 0.0)
    b = np.array([-(dx * dx) * d[j, i] for (j, i) in cells])
    ref = np.linalg.solve(A_bf, b)
    sol = SV.exact_solve(P, d, dx)
    assert np.allclose([sol[j, i] for (j, i) in cells], ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("seed", range(4))
def test_matrix_spd_symmetric(seed):
    rng = np.random.default_rng(seed)
    flags = random_mask(rng, 12, 10, p=0.3)
    P = G.plan(flags)
    A, _ = G.assemble(P)
    Ad = A.toarray()
    assert np.array_equal(Ad, Ad.T)
    assert np.array_equal(np.diag(Ad), P.k[P.fluid])
    ev = np.linalg.eigvalsh(Ad)
    assert ev.min() > 0  # every fluid component touches the open row
    # eigenvalues of L = -A/dx^2 are strictly negative


def test_enclosed_pocket_would_be_singular():
    # a ring of solid cells encloses fluid; without the pocket fill the
    # enclosed block would be a singular Neumann problem
    flags = np.zeros((9, 9), dtype=np.uint8)
    flags[2, 2:7] = 1; flags[6, 2:7] = 1; flags[2:7, 2] = 1; flags[2:7, 6] = 1
    P = G.plan(flags)
    assert not P.fluid[4, 4] and not P.fluid[3:6, 3:6].any()
    A, _ = G.assemble(P)
    assert np.linalg.eigvalsh(A.toarray()).min() > 0


# ---- invariants of the projection ------------------------------------------

@pytest.mark.parametrize("seed", range(3))
def test_divergence_free_after_exact_projection(seed):
    sc = scenes.plume_scene(32, seed=seed, n_obstacles=2)
    u, v = scenes.random_faces(32, 32, seed, kind="mixed")
    P = G.plan(sc.flags)
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, sc.dx)
    phi = SV.exact_solve(P, d, sc.dx)
    u2, v2 = G.correct(P, u, v, phi, sc.dx)
    d2 = G.divergence(P, u2, v2, sc.dx)
    assert np.abs(d2).max() <= 1e-12 * np.abs(d).max()
    # the residual identity div(u - grad phi) = d - L phi holds for any phi
    psi = np.where(P.fluid, np.random.default_rng(seed).standard_normal(P.shape), 0)
    u3, v3 = G.correct(P, u, v, psi, sc.dx)
    assert np.allclose(G.divergence(P, u3, v3, sc.dx), G.residual(P, d, psi, sc.dx),
                       atol=1e-10 * np.abs(d).max())


def test_DT_equals_minus_G():
    rng = np.random.default_rng(3)
    sc = scenes.plume_scene(24, seed=5, n_obstacles=2)
    P = G.plan(sc.flags)
    u = rng.standard_normal((24, 25)); v = rng.standard_normal((25, 24))
    u, v = G.enforce_bc(P, u, v)
    v[0, :] = 0.0  # inflow faces are data, not unknowns
    phi = np.where(P.fluid, rng.standard_normal(P.shape), 0.0)
    dx = sc.dx
    d = G.divergence(P, u, v, dx)
    gu, gv = G.correct(P, np.zeros_like(u), np.zeros_like(v), phi, dx)  # = -grad phi
    lhs = np.sum(d * phi)
    rhs = np.sum(u * gu) + np.sum(v * gv)  # = -<u, grad phi>
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1)


def test_mirror_equivariance():
    # no obstacles: mirroring x maps the problem onto itself with u -> -u
    n = 32
    sc = scenes.plume_scene(n, seed=0, n_obstacles=0)
    assert np.array_equal(sc.flags, sc.flags[:, ::-1])
    u, v = scenes.random_faces(n, n, 4, kind="mixed")
    P = G.plan(sc.flags)

    def solve(u, v):
        u, v = G.enforce_bc(P, u, v)
        return SV.exact_solve(P, G.divergence(P, u, v, sc.dx), sc.dx)

    ex1 = solve(u, v)
    ex2 = solve(-u[:, ::-1], v[:, ::-1])
    assert np.allclose(ex2, ex1[:, ::-1], atol=1e-13 * np.abs(ex1).max())


def test_idempotence():
    sc = scenes.plume_scene(32, seed=1, n_obstacles=1)
    u, v = scenes.random_faces(32, 32, 9)
    P = G.plan(sc.flags)
    u, v = G.enforce_bc(P, u, v)
    d = G.divergence(P, u, v, sc.dx)
    u2, v2 = G.correct(P, u, v, SV.exact_solve(P, d, sc.dx), sc.dx)
    r = PR.project(sc.flags, u2, v2, sc.dx, method="jacobi", threshold=1e-9)
    assert r["iters"] == 0
    assert np.abs(r["phi"]).max() == 0.0
    assert np.allclose(r["u"], u2) and np.allclose(r["v"], v2)


def test_inflow_faces_untouched_and_walls_zero():
    sc = scenes.plume_scene(32, seed=2, n_obstacles=1)
    u, v = scenes.random_faces(32, 32, 2)
    r = PR.project(sc.flags, u, v, sc.dx, method="pcg", threshold=1e-8)
    P = r["plan"]
    assert np.array_equal(r["v"][0][P.vinflow], v[0][P.vinflow])
    assert np.all(r["v"][0][~P.vinflow] == 0)
    assert np.all(r["u"][:, 0] == 0) and np.all(r["u"][:, -1] == 0)
    assert np.all(r["u"][~P.uopen] == 0)
