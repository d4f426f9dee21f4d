"""GPU parity of the full time step (CFL dt, MacCormack advection, buoyancy,
inflow, boundary faces, projection) against the FP64 oracle.  The plume is
chaotic, so parity is per step: the oracle re-steps from the GPU's state."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import advect as AD
from oracle import grid as G
from oracle import project as PR
from tests.gpu_util import to_dev, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def close_mostly(a, b, tol, frac=0.999):
    """All but a tiny fraction of points agree to `tol` (relative to the field
    scale): the MacCormack limiter switches its bounds discontinuously, so a
    position rounded differently in FP32 may pick another bound pair."""
    scale = max(np.abs(b).max(), 1e-30)
    ok = np.abs(a - b) <= tol * scale
    return ok.mean() >= frac


@pytest.mark.parametrize("n,nobs,seed,method", [(64, 0, 0, "jacobi"), (128, 2, 1, "pcg"),
                                                 (96, 1, 2, "jacobi")])
def test_step_parity_per_step(n, nobs, seed, method):
    say("step", n, nobs, method)
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    P = G.plan(sc.flags)
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device="cuda")
    u = torch.zeros((n, n + 1), dtype=torch.float32, device="cuda")
    v = torch.zeros((n + 1, n), dtype=torch.float32, device="cuda")
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    fixed = 30 if method == "jacobi" else 0
    for step in range(8):
        xi = scenes.inflow_noise(seed, step, n)
        r0 = rho.cpu().numpy().astype(np.float64)
        u0 = u.cpu().numpy().astype(np.float64)
        v0 = v.cpu().numpy().astype(np.float64)
        pr.step_async(rho, u, v, tf, p, to_dev(xi), threshold=1e-3, g=sc.g, drho=sc.drho,
                      u_in=sc.u_in, method=method, fixed_iters=fixed, max_iters=20000)
        torch.cuda.synchronize()
        res = pr.result()
        dt_o = AD.cfl_dt(u0, v0, sc.dx, sc.u_in)
        assert res.dt == pytest.approx(dt_o, rel=1e-12)
        xi32 = np.float32(xi).astype(np.float64)
        ro, us, vs = AD.advect_step(P, sc.flags, r0, u0, v0, sc.dx, res.dt, sc.g, sc.rho0,
                                    sc.drho, sc.u_in, xi32)
        assert close_mostly(rho.cpu().numpy(), ro, 1e-5)
        if method == "jacobi":
            o = PR.project(sc.flags, us, vs, sc.dx, dt=res.dt, method="jacobi", fixed_iters=fixed)
            assert res.iters == fixed
        else:
            o = PR.project(sc.flags, us, vs, sc.dx, dt=res.dt, method="pcg", threshold=1e-3)
            assert abs(res.iters - o["iters"]) <= max(3, 0.1 * o["iters"])
            assert res.e1_final < 1.05e-3
        assert close_mostly(u.cpu().numpy(), o["u"], 1e-4)
        assert close_mostly(v.cpu().numpy(), o["v"], 1e-4)
        assert res.e1_init == pytest.approx(o["e1_init"], rel=1e-2)
        say("  step", step, "dt", res.dt, "iters", res.iters, "e1_init", res.e1_init)


def test_step_bad_arguments():
    pr = hp.Projector(32, 32, 1 / 32)
    t = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        pr.step_async(t, t, t, t, t, t, 1e-3, g=1.0, drho=0.01)
