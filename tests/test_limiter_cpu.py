"""CPU checks of the limiter-ambiguity helper used by the GPU time-step
parity: perturbing the back-trace positions by less than the rounding
allowance changes the oracle's advection only at flagged points, and only
to one of their limiter candidates."""
import numpy as np
import pytest

import scenes
from oracle import advect as AD
from oracle import grid as G
from tests import limiter as LM


@pytest.mark.parametrize("n,seed,tiny", [(48, 0, False), (64, 1, False), (64, 1, True)])
def test_perturbed_positions_change_only_flagged_points(n, seed, tiny, monkeypatch):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1)
    P = G.plan(sc.flags)
    rho = scenes.random_density(n, n, seed, sc.rho0, 0.2)
    u, v = (0.5 * a for a in scenes.random_faces(n, n, seed, kind="smooth"))
    if tiny:
        # velocities far below a cell per step over most of the grid (a plume
        # shortly after the start): most back-traces sit on grid lines
        u = u * np.where(np.arange(n + 1)[None, :] < n // 2, 1e-9, 1.0)
        v = v * 1e-9
    u, v = G.enforce_bc(P, u, v)
    dt = AD.cfl_dt(u, v, sc.dx, sc.u_in)
    xi = np.zeros(n)
    ref = AD.advect_step(P, sc.flags, rho, u, v, sc.dx, dt, sc.g, sc.rho0, 0.2, sc.u_in, xi)
    eps = LM.position_eps(n + 1, n + 1)
    rng = np.random.default_rng(seed)
    real = AD._sample

    def jittered(q, X, Y):
        # every position moved by up to half the allowance, as FP32 rounding might
        return real(q, X + rng.uniform(-0.5, 0.5, X.shape) * eps,
                    Y + rng.uniform(-0.5, 0.5, Y.shape) * eps)

    monkeypatch.setattr(AD, "_sample", jittered)
    out = AD.advect_step(P, sc.flags, rho, u, v, sc.dx, dt, sc.g, sc.rho0, 0.2, sc.u_in, xi)
    monkeypatch.setattr(AD, "_sample", real)
    # the jitter moves continuous samples by |grad q| eps; only limiter flips are discrete
    rep = LM.compare_advected(P, rho, u, v, dt, sc.dx, sc.g, sc.rho0, out, ref, tol=1e-5)
    for name, r in rep.items():
        assert r["n_bad"] == 0, (name, r)
        assert r["n_flipped"] <= r["n_amb"]
    if tiny:  # the jitter did flip limiter choices, and each matched a candidate
        assert sum(r["n_flipped"] for r in rep.values()) > 10


def test_flags_points_on_grid_lines():
    X = np.array([[3.0, 3.0 + 1e-9, 2.5, 0.0, 7.0]])
    Y = np.array([[1.5, 1.5, 2.0 - 1e-9, 1.5, 1.5]])
    amb = LM.ambiguous(X, Y, 10, 8, 1e-6)
    assert amb.tolist() == [[True, True, True, False, False]]
