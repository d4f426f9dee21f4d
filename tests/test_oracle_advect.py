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
