"""Pins of the oracle's advection/force step (Sec. 2.2: MacCormack
semi-Lagrangian advection, forward-Euler buoyancy)."""
import numpy as np
import pytest

from oracle import advect as AD
from oracle import grid as G
import scenes


def test_zero_velocity_is_identity():
    rng = np.random.default_rng(0)
    q = rng.standard_normal((10, 12))
    z = np.zeros_like(q)
    assert np.array_equal(AD.maccormack(q, z, z, 0.3), q)


@pytest.mark.parametrize("sx,sy", [(1, 0), (0, 2), (-1, 1), (2, -3)])
def test_integer_shift_is_exact(sx, sy):
    rng = np.random.default_rng(1)
    q = rng.standard_normal((16, 16))
    vx = np.full_like(q, float(sx)); vy = np.full_like(q, float(sy))
    out = AD.maccormack(q, vx, vy, 1.0)
    # interior points whose forward and backward traces stay inside the grid
    m = 4
    ref = np.roll(np.roll(q, sy, axis=0), sx, axis=1)
    assert np.allclose(out[m:-m, m:-m], ref[m:-m, m:-m], atol=1e-14)


def test_linear_field_translated_exactly():
    # bilinear interpolation is exact on a linear field, so SL and the
    # MacCormack correction both translate it exactly (away from the clamp)
    H, W = 20, 24
    J, I = np.mgrid[0:H, 0:W].astype(np.float64)
    q = 0.3 * I - 0.7 * J + 2.0
    vx = np.full_like(q, 0.37); vy = np.full_like(q, -0.21)
    out = AD.maccormack(q, vx, vy, 1.0)
    ref = 0.3 * (I - 0.37) - 0.7 * (J + 0.21) + 2.0
    m = 3
    assert np.allclose(out[m:-m, m:-m], ref[m:-m, m:-m], atol=1e-13)


def test_maccormack_within_local_extrema():
    rng = np.random.default_rng(2)
    q = rng.standard_normal((24, 24))
    vx = rng.uniform(-1.5, 1.5, q.shape); vy = rng.uniform(-1.5, 1.5, q.shape)
    out = AD.maccormack(q, vx, vy, 0.8)
    J, I = np.mgrid[0:24, 0:24].astype(np.float64)
    _, mn, mx = AD._sample(q, I - 0.8 * vx, J - 0.8 * vy)
    assert np.all(out >= mn - 1e-15) and np.all(out <= mx + 1e-15)


def test_buoyancy_closed_form():
    # uniform density deficit, fluid at rest, no obstacles: after one step
    # every interior/top v-face gains exactly dt g drho (rho0 = 1)
    n = 16
    sc = scenes.plume_scene(n, seed=0, n_obstacles=0, drho=0.01, ri=0.1)
    P = G.plan(sc.flags)
    rho = np.full((n, n), 1.0 - 0.25)
    u = np.zeros((n, n + 1)); v = np.zeros((n + 1, n))
    dt = 0.01
    rho_n, us, vs = AD.advect_step(P, sc.flags, rho, u, v, sc.dx, dt, sc.g, 1.0, sc.drho,
                                   sc.u_in, np.zeros(n))
    assert np.allclose(vs[1:], dt * sc.g * 0.25, rtol=1e-15)
    assert np.all(us == 0)
    assert np.allclose(vs[0][P.vinflow], sc.u_in) and np.all(vs[0][~P.vinflow] == 0)


def test_richardson_reading_reproduces_paper_plume():
    # Sec. 4.1 prints Ri = 14.8 for drho = 0.01, U = 0.01 m/s, g = 0.002 m/s^2
    # and an inlet radius R = 74.25 m (L = 512 m); with R as the length in
    # Eq. (1) these give Ri = 14.85, and 2R/L = 0.29 is the D_in of Sec. 2.1.
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_plume.json")))
    ri = gold["drho"] * gold["g"] * gold["R"] / gold["U"] ** 2
    assert ri == pytest.approx(gold["Ri"], abs=0.06)
    assert 2 * gold["R"] / gold["L"] == pytest.approx(gold["D_in_over_L"], abs=1e-3)
    g = scenes.gravity_from_richardson(ri, gold["U"], gold["drho"], 2 * gold["R"])
    assert g == pytest.approx(gold["g"], rel=1e-12)


def test_cfl_dt():
    u = np.zeros((4, 5)); v = np.zeros((5, 4)); v[2, 1] = -3.0
    assert AD.cfl_dt(u, v, 0.25, 1.0) == pytest.approx(0.5 * 0.25 / 3.0)
    assert AD.cfl_dt(0 * u, 0 * v, 0.25, 1.0) == pytest.approx(0.125)


# ---- staggered-velocity reconstruction (Sec. 2.2: the velocity is advected
# like the density, so every sample point of every field needs both velocity
# components at its own position on the MAC grid).  Positions below are in
# cell units: centre (i + 1/2, j + 1/2), u face (i, j + 1/2), v face
# (i + 1/2, j).  Averages of a linear field are exact at the mean position,
# so linear face velocities must come back exactly wherever the stencil is
# away from a wall; at a wall the missing column (row) is replaced by the
# nearest one that exists (positions clamped to the grid).

def _linear_faces(nx, ny, cu, cv):
    """u and v sampled from the linear functions cu(X, Y), cv(X, Y) at their
    face positions."""
    Ju, Iu = np.mgrid[0:ny, 0:nx + 1].astype(np.float64)
    Jv, Iv = np.mgrid[0:ny + 1, 0:nx].astype(np.float64)
    return cu(Iu, Ju + 0.5), cv(Iv + 0.5, Jv)


def test_velocity_reconstruction_is_exact_for_linear_fields():
    nx, ny = 7, 5  # rectangular: a transposed index fails
    cu = lambda X, Y: 0.3 + 0.7 * X - 1.1 * Y
    cv = lambda X, Y: -0.2 + 1.3 * X + 0.4 * Y
    u, v = _linear_faces(nx, ny, cu, cv)
    # cell centres
    J, I = np.mgrid[0:ny, 0:nx].astype(np.float64)
    ux, vy = AD._vel_at_centres(u, v)
    assert np.allclose(ux, cu(I + 0.5, J + 0.5), rtol=0, atol=1e-14)
    assert np.allclose(vy, cv(I + 0.5, J + 0.5), rtol=0, atol=1e-14)
    # u faces: v interpolated at (i, j + 1/2); interior columns exact
    uu, vv = AD._vel_at_ufaces(u, v)
    assert np.array_equal(uu, u)
    Ju, Iu = np.mgrid[0:ny, 0:nx + 1].astype(np.float64)
    assert np.allclose(vv[:, 1:nx], cv(Iu, Ju + 0.5)[:, 1:nx], rtol=0, atol=1e-14)
    # walls: the clamped stencil is the mean of the one column that exists
    assert np.allclose(vv[:, 0], cv(0.5, np.arange(ny) + 0.5), rtol=0, atol=1e-14)
    assert np.allclose(vv[:, nx], cv(nx - 0.5, np.arange(ny) + 0.5), rtol=0, atol=1e-14)
    # v faces: u interpolated at (i + 1/2, j); interior rows exact
    uv, vv2 = AD._vel_at_vfaces(u, v)
    assert np.array_equal(vv2, v)
    Jv, Iv = np.mgrid[0:ny + 1, 0:nx].astype(np.float64)
    assert np.allclose(uv[1:ny], cu(Iv + 0.5, Jv)[1:ny], rtol=0, atol=1e-14)
    assert np.allclose(uv[0], cu(np.arange(nx) + 0.5, 0.5), rtol=0, atol=1e-14)
    assert np.allclose(uv[ny], cu(np.arange(nx) + 0.5, ny - 0.5), rtol=0, atol=1e-14)


def _maccormack_closed_form(q, vel, r, X, Y, H, W, at):
    """MacCormack (Sec. 2.2) of a linear field q with a velocity field vel
    (both functions of the position), evaluated at positions (X, Y): the
    back-trace, the forward trace of the back-traced field and the
    correction, each exact for linear data; then the limiter bounds, the
    extremes of q on the four grid points around the back-trace point.
    `at` maps a position to the sampled array's index coordinates."""
    ux, vy = vel(X, Y)
    qhat = lambda X_, Y_: q(X_ - r * vel(X_, Y_)[0], Y_ - r * vel(X_, Y_)[1])
    q_hat = qhat(X, Y)
    q_til = qhat(X + r * ux, Y + r * vy)
    q_new = q_hat + 0.5 * (q(X, Y) - q_til)
    bi, bj = at(X - r * ux, Y - r * vy)
    i0 = np.floor(bi); j0 = np.floor(bj)
    ox, oy = X - at(X, Y)[0], Y - at(X, Y)[1]  # index -> position offset
    corners = [q(i0 + di + ox, j0 + dj + oy) for di in (0, 1) for dj in (0, 1)]
    mn = np.minimum.reduce(corners); mx = np.maximum.reduce(corners)
    inside = (bi > 0) & (bi < W - 1) & (bj > 0) & (bj < H - 1)
    return np.clip(q_new, mn, mx), inside


def test_advect_step_closed_form_with_linear_velocity():
    """Whole advect_step on linear, divergence-free face velocities
    u = U0 + b Y, v = V0 + e X and a linear density: the back-traced fields
    stay linear, so every point away from the walls and the inflow row has
    a closed form; a wrong neighbour in a face reconstruction shifts the
    velocity by e/2 or b/2 and fails here."""
    n = 32
    sc = scenes.plume_scene(n, seed=0, n_obstacles=0)
    P = G.plan(sc.flags)
    U0, b, V0, e = 0.31, 0.023, 0.27, -0.017  # cells per unit time
    cu = lambda X, Y: U0 + b * Y + 0 * X
    cv = lambda X, Y: V0 + e * X + 0 * Y
    vel = lambda X, Y: (cu(X, Y), cv(X, Y))
    crho = lambda X, Y: 1.0 + 0.013 * X - 0.009 * Y
    dx = sc.dx
    u, v = _linear_faces(n, n, lambda X, Y: cu(X, Y) * dx, lambda X, Y: cv(X, Y) * dx)
    J, I = np.mgrid[0:n, 0:n].astype(np.float64)
    rho = crho(I + 0.5, J + 0.5)
    dt = 1.7  # velocities in cells per unit time: back-trace offsets of about half a cell
    rho_n, us, vs = AD.advect_step(P, sc.flags, rho, u, v, dx, dt, 0.0, sc.rho0, sc.drho,
                                   sc.u_in, np.zeros(n))
    m = 4
    # density at the centres
    ref, ok = _maccormack_closed_form(crho, vel, dt, I + 0.5, J + 0.5, n, n,
                                      lambda X, Y: (X - 0.5, Y - 0.5))
    sel = ok.copy(); sel[:m] = sel[-m:] = False; sel[:, :m] = sel[:, -m:] = False
    assert sel.sum() > 300
    assert np.allclose(rho_n[sel], ref[sel], rtol=0, atol=1e-13)
    # u at the u faces (values in physical units: closed form times dx)
    Ju, Iu = np.mgrid[0:n, 0:n + 1].astype(np.float64)
    ref, ok = _maccormack_closed_form(cu, vel, dt, Iu, Ju + 0.5, n, n + 1,
                                      lambda X, Y: (X, Y - 0.5))
    sel = ok.copy(); sel[:m] = sel[-m:] = False; sel[:, :m] = sel[:, -m:] = False
    assert np.allclose(us[sel], dx * ref[sel], rtol=0, atol=1e-15)
    # v at the v faces
    Jv, Iv = np.mgrid[0:n + 1, 0:n].astype(np.float64)
    ref, ok = _maccormack_closed_form(cv, vel, dt, Iv + 0.5, Jv, n + 1, n,
                                      lambda X, Y: (X - 0.5, Y))
    sel = ok.copy(); sel[:m] = sel[-m:] = False; sel[:, :m] = sel[:, -m:] = False
    assert np.allclose(vs[sel], dx * ref[sel], rtol=0, atol=1e-15)


@pytest.mark.parametrize("which", ["ufaces_shift", "vfaces_shift", "centres_swap"])
def test_reconstruction_pin_detects_a_wrong_neighbour(which, monkeypatch):
    """The closed-form pin above fails for a plausible indexing mistake in
    any of the three reconstructions (mistakes planted in the oracle here,
    on the CPU)."""
    nx = 7
    if which == "ufaces_shift":
        def bad(u, v):
            ny, nx1 = u.shape
            il = np.clip(np.arange(nx1), 0, nx1 - 2)
            ir = np.clip(np.arange(nx1) + 1, 0, nx1 - 2)
            return u, 0.25 * (v[:-1, il] + v[:-1, ir] + v[1:, il] + v[1:, ir])
        monkeypatch.setattr(AD, "_vel_at_ufaces", bad)
    elif which == "vfaces_shift":
        def bad(u, v):
            ny1, nx_ = v.shape
            jb = np.clip(np.arange(ny1), 0, ny1 - 2)
            jt = np.clip(np.arange(ny1) + 1, 0, ny1 - 2)
            return 0.25 * (u[jb, :-1] + u[jb, 1:] + u[jt, :-1] + u[jt, 1:]), v
        monkeypatch.setattr(AD, "_vel_at_vfaces", bad)
    else:
        def bad(u, v):
            return 0.5 * (v[:-1, :] + v[1:, :]), 0.5 * (u[:, :-1] + u[:, 1:])
        monkeypatch.setattr(AD, "_vel_at_centres", bad)
    with pytest.raises(AssertionError):
        test_advect_step_closed_form_with_linear_velocity()


def test_inflow_density_reset_only_on_open_inflow_cells():
    """The injected light fluid enters through the prescribed inflow faces
    (Sec. 2.1): the density reset covers the row-0 cells whose bottom face is
    an inflow face of the plan (fluid cells flagged inflow), and a solid
    cell flagged inflow keeps its value."""
    n = 16
    sc = scenes.plume_scene(n, seed=0, n_obstacles=0)
    flags = sc.flags.copy()
    inflow = np.nonzero(flags[0] & G.FLAG_INFLOW)[0]
    assert inflow.size >= 2
    flags[0, inflow[0]] |= G.FLAG_SOLID
    P = G.plan(flags)
    rho = np.full((n, n), 0.5)
    z_u = np.zeros((n, n + 1)); z_v = np.zeros((n + 1, n))
    rho_n, _, vs = AD.advect_step(P, flags, rho, z_u, z_v, sc.dx, 1e-3, 0.0, 1.0, 0.2, 1.0,
                                  np.zeros(n))
    assert rho_n[0, inflow[0]] == 0.5 and vs[0, inflow[0]] == 0.0
    assert np.all(rho_n[0, inflow[1:]] == 0.8) and np.all(vs[0, inflow[1:]] == 1.0)
    others = np.setdiff1d(np.arange(n), inflow)
    assert np.all(rho_n[0, others] == 0.5)
