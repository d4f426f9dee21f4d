"""GPU parity of the time step (CFL dt, MacCormack advection, buoyancy,
inflow, boundary faces, projection; Sec. 2.2) against the FP64 oracle,
element by element.

The advection half is compared point by point on the same FP32-rounded
inputs.  Only points whose back-trace lands within FP32 rounding of a grid
line may differ (the limiter's sample cell is a discrete choice there; see
tests/limiter.py), and each of those must equal one of the values the
limiter gives for the sample cells within rounding of the back-trace.  Inflow and wall faces must match exactly.  The projection
half is compared on the GPU's own u* (the advection is deterministic, so a
separate advection call reproduces what the step projected), element-wise
at fixed iteration counts.  A rollout is checked step by step: the oracle
re-steps from the GPU's state at the start of every step (the plume is
chaotic, so two independent trajectories are not comparable)."""
import os

import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import advect as AD
from oracle import grid as G
from oracle import project as PR
from tests.gpu_util import to_dev, f32, rel_l2
from tests import limiter as LM

pytestmark = pytest.mark.gpu

ADV_TOL = 1e-5    # advected fields, relative to the field's max (FP32 vs FP64)
PROJ_TOL = 1e-5   # projected faces and pressure at fixed iterations
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_2109_09363_amd", "weights", "plume_s4c64.npy")


def say(*a):
    print(*a, flush=True)


def np64(t):
    return t.cpu().numpy().astype(np.float64)


def seeded_state(n, seed, drho=0.2):
    rho = f32(scenes.random_density(n, n, seed, 1.0, drho))
    u, v = (f32(0.5 * a) for a in scenes.random_faces(n, n, seed, kind="smooth"))
    return rho, u, v


def gpu_advect(pr, rho, u, v, xi, sc, drho):
    tr, tu, tv = to_dev(rho), to_dev(u), to_dev(v)
    pr.advect_async(tr, tu, tv, to_dev(xi), g=sc.g, drho=drho, u_in=sc.u_in)
    torch.cuda.synchronize()
    return np64(tr), np64(tu), np64(tv)


def check_advection(P, sc, rho, u, v, xi, drho, dt, gpu_out, label):
    """Element-wise comparison of one advection + force step."""
    ref = AD.advect_step(P, sc.flags, rho, u, v, sc.dx, dt, sc.g, sc.rho0, drho, sc.u_in, xi)
    rep = LM.compare_advected(P, rho, u, v, dt, sc.dx, sc.g, sc.rho0, gpu_out, ref, ADV_TOL)
    say(f"  {label}: " + ", ".join(f"{k} max rel {r['max_rel_clear']:.1e} ({r['n_flipped']} "
                                   f"limiter flips, {r['n_amb']} ambiguous of {r['n']})"
                                   for k, r in rep.items()))
    for k, r in rep.items():
        assert r["n_bad"] == 0, (k, r)
    rg, ug, vg = gpu_out
    # inflow and wall faces exactly (the prescribed values are FP32 roundings)
    assert np.array_equal(vg[0], f32(ref[2][0]))
    assert np.all(ug[:, 0] == 0) and np.all(ug[:, -1] == 0)
    assert np.all(ug[~P.uopen] == 0) and np.all(vg[1:][~P.vopen[1:]] == 0)
    assert np.array_equal(rg[0][P.vinflow], f32(ref[0][0][P.vinflow]))
    return ref


@pytest.mark.parametrize("n,nobs,seed", [(64, 1, 10), (256, 2, 11), (512, 3, 12)])
def test_advection_parity_elementwise(n, nobs, seed):
    say("advection", n, nobs, seed)
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    P = G.plan(sc.flags)
    rho, u, v = seeded_state(n, seed)
    u, v = G.enforce_bc(P, u, v)
    xi = f32(scenes.inflow_noise(seed, 0, n))
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0)
    pr.plan(to_dev(sc.flags, torch.uint8))
    out = gpu_advect(pr, rho, u, v, xi, sc, 0.2)
    # the device takes max |u|, max |v| of the same FP32 values and divides in
    # FP64, so its dt is the oracle's (the step tests check res.dt)
    dt = AD.cfl_dt(u, v, sc.dx, sc.u_in)
    check_advection(P, sc, rho, u, v, xi, 0.2, dt, out, f"{n}^2")


@pytest.mark.parametrize("n,nobs,seed,method,fixed", [(96, 2, 11, "pcg", 40), (256, 1, 13, "jacobi", 64),
                                                       (128, 2, 14, "jacobi", 24)])
def test_step_parity_elementwise(n, nobs, seed, method, fixed):
    """One full hyp_step: its advected density equals the advection call's
    bit for bit, and its projection of that u* matches the oracle's
    projection of the same u* point by point."""
    say("step", n, nobs, seed, method, fixed)
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    P = G.plan(sc.flags)
    rho, u, v = seeded_state(n, seed)
    xi = f32(scenes.inflow_noise(seed, 1, n))
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    r_a, u_a, v_a = gpu_advect(pr, rho, u, v, xi, sc, 0.2)
    tr, tu, tv = to_dev(rho), to_dev(u), to_dev(v)
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    pr.step_async(tr, tu, tv, tf, p, to_dev(xi), threshold=0.0, g=sc.g, drho=0.2, u_in=sc.u_in,
                  method=method, fixed_iters=fixed)
    torch.cuda.synchronize()
    res = pr.result()
    assert res.status == 0 and res.iters == fixed
    assert np.array_equal(np64(tr), r_a)
    check_advection(P, sc, rho, u, v, xi, 0.2, res.dt, (r_a, u_a, v_a), "advection")
    o = PR.project(sc.flags, u_a, v_a, sc.dx, dt=res.dt, method=method, fixed_iters=fixed)
    ug, vg, pg = np64(tu), np64(tv), np64(p)
    eu = np.abs(ug - o["u"]).max() / np.abs(o["u"]).max()
    ev = np.abs(vg - o["v"]).max() / np.abs(o["v"]).max()
    ep = np.abs(pg - o["p"]).max() / np.abs(o["p"]).max()
    say(f"  projection of u*: max rel u {eu:.1e} v {ev:.1e} p {ep:.1e}; e1_init "
        f"{res.e1_init:.6e} vs {o['e1_init']:.6e}")
    assert eu <= PROJ_TOL and ev <= PROJ_TOL and ep <= PROJ_TOL
    assert res.e1_init == pytest.approx(o["e1_init"], rel=1e-5)
    assert res.e1_final == pytest.approx(o["e1_final"], rel=1e-3)


def test_benchmark_step_512():
    """The benchmark's own step: 512^2 plume (0-3 disks, seed 0) developed
    by five PCG-projected steps from rest on the GPU, then one step with the
    4-scale 64-channel BF16 network and Jacobi to mean|div| < 1e-3, E_1
    tested every 768 sweeps."""
    if not os.path.exists(WEIGHTS):
        pytest.skip("trained weights not present")
    n = 512
    sc = scenes.plume_scene(n, seed=0, n_obstacles=(0, 3))
    P = G.plan(sc.flags)
    w = np.load(WEIGHTS, allow_pickle=False).astype(np.float32)
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0, 4, 64, "bf16")
    tw = to_dev(w)
    pr.set_weights(tw)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device="cuda")
    u = torch.zeros((n, n + 1), dtype=torch.float32, device="cuda")
    v = torch.zeros((n + 1, n), dtype=torch.float32, device="cuda")
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    for s in range(5):
        pr.step_async(rho, u, v, tf, p, to_dev(f32(scenes.inflow_noise(0, s, n))), 1e-3, g=sc.g,
                      drho=sc.drho, u_in=sc.u_in, method="pcg", max_iters=1000000, check_every=1)
    torch.cuda.synchronize()
    rho0_, u0_, v0_ = np64(rho), np64(u), np64(v)
    xi = f32(scenes.inflow_noise(0, 5, n))
    r_a, u_a, v_a = gpu_advect(pr, rho0_, u0_, v0_, xi, sc, sc.drho)
    pr.step_async(rho, u, v, tf, p, to_dev(xi), 1e-3, g=sc.g, drho=sc.drho, u_in=sc.u_in,
                  method="hybrid", max_iters=1000000, check_every=768)
    torch.cuda.synchronize()
    res = pr.result()
    say("  benchmark step: sweeps", res.iters, "status", res.status, "e1", res.e1_final)
    assert res.status == 0 and res.e1_final < 1e-3
    assert np.array_equal(np64(rho), r_a)
    check_advection(P, sc, rho0_, u0_, v0_, xi, sc.drho, res.dt, (r_a, u_a, v_a), "advection")
    o = PR.project(sc.flags, u_a, v_a, sc.dx, dt=res.dt, threshold=1e-3, method="hybrid", params=w,
                   S=4, C=64, bf16=True, check_every=768, max_iters=1000000)
    say("  oracle sweeps", o["iters"])
    assert abs(res.iters - o["iters"]) <= 768
    of = PR.project(sc.flags, u_a, v_a, sc.dx, dt=res.dt, method="hybrid", params=w, S=4, C=64,
                    bf16=True, fixed_iters=res.iters) if res.iters != o["iters"] else o
    ug, vg, pg = np64(u), np64(v), np64(p)
    err_p = rel_l2(pg, of["p"], P.fluid)
    eu = np.abs(ug - of["u"]).max() / np.abs(of["u"]).max()
    ev = np.abs(vg - of["v"]).max() / np.abs(of["v"]).max()
    say(f"  at the GPU's sweep: rel L2 p {err_p:.1e}, max rel u {eu:.1e} v {ev:.1e}")
    assert err_p <= 1e-3
    assert eu <= 1e-4 and ev <= 1e-4


@pytest.mark.parametrize("n,nobs,seed,method", [(64, 0, 0, "jacobi"), (128, 2, 1, "pcg"),
                                                 (96, 1, 2, "jacobi")])
def test_rollout_parity_per_step(n, nobs, seed, method):
    """Eight steps of the plume from rest on the GPU; before every step the
    oracle takes the GPU's state and re-steps it: the advection point by
    point, and the projection at the same fixed sweep count (Jacobi) or with
    its own stop (PCG: iterations within 10 %, and no farther from the exact
    solve of the GPU's u* than the oracle's stopped iterate)."""
    say("rollout", n, nobs, method)
    from oracle import solve as SV
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
        xi = f32(scenes.inflow_noise(seed, step, n))
        r0, u0, v0 = np64(rho), np64(u), np64(v)
        r_a, u_a, v_a = gpu_advect(pr, r0, u0, v0, xi, sc, sc.drho)
        pr.step_async(rho, u, v, tf, p, to_dev(xi), threshold=1e-3, g=sc.g, drho=sc.drho,
                      u_in=sc.u_in, method=method, fixed_iters=fixed, max_iters=20000)
        torch.cuda.synchronize()
        res = pr.result()
        assert res.dt == pytest.approx(AD.cfl_dt(u0, v0, sc.dx, sc.u_in), rel=1e-12)
        assert np.array_equal(np64(rho), r_a)
        check_advection(P, sc, r0, u0, v0, xi, sc.drho, res.dt, (r_a, u_a, v_a), f"step {step}")
        ug, vg, pg = np64(u), np64(v), np64(p)
        if method == "jacobi":
            o = PR.project(sc.flags, u_a, v_a, sc.dx, dt=res.dt, method="jacobi", fixed_iters=fixed)
            assert res.iters == fixed
            for a, b in ((ug, o["u"]), (vg, o["v"]), (pg, o["p"])):
                assert np.abs(a - b).max() <= PROJ_TOL * max(np.abs(b).max(), 1e-30)
        else:
            o = PR.project(sc.flags, u_a, v_a, sc.dx, dt=res.dt, method="pcg", threshold=1e-3)
            assert abs(res.iters - o["iters"]) <= max(3, 0.1 * o["iters"])
            assert res.status == 0 and res.e1_final < 1e-3
            uu, vv = G.enforce_bc(P, u_a, v_a)
            ex = sc.rho0 / res.dt * SV.exact_solve(P, G.divergence(P, uu, vv, sc.dx), sc.dx)
            eg, eo = rel_l2(pg, ex, P.fluid), rel_l2(o["p"], ex, P.fluid)
            say(f"    iters {res.iters} / {o['iters']}, p from exact: gpu {eg:.1e} oracle {eo:.1e}")
            # a threshold-stopped CG iterate is as far from the exact solve as
            # the stop allows: the GPU's may be no farther than the oracle's
            assert eg <= 1.5 * eo + 1e-4
        assert res.e1_init == pytest.approx(o["e1_init"], rel=1e-5)


def test_step_bad_arguments():
    pr = hp.Projector(32, 32, 1 / 32)
    t = torch.zeros((32, 32), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        pr.step_async(t, t, t, t, t, t, 1e-3, g=1.0, drho=0.01)


@pytest.mark.parametrize("method", ["hybrid", "pcg"])
def test_captured_step_replays_match_eager_steps(method):
    """A time step captured as a hipGraph (torch.cuda.graph around the
    library call: the persistent solver becomes a plain launch of the same
    grid) and replayed with a new inflow noise each time, with eager work
    and synchronisations between the replays: every replay's state and
    result equal those of the eager step from the same state, bit for bit."""
    n = 256
    sc = scenes.plume_scene(n, seed=21, n_obstacles=2)
    w = torch.from_numpy(np.load(WEIGHTS, allow_pickle=False).astype(np.float32)).cuda()
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0, 4, 64, "bf16")
    pr.set_weights(w)
    flags = to_dev(sc.flags, torch.uint8)
    pr.plan(flags)
    rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device="cuda")
    u = torch.zeros((n, n + 1), dtype=torch.float32, device="cuda")
    v = torch.zeros((n + 1, n), dtype=torch.float32, device="cuda")
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    xb = torch.empty((n,), dtype=torch.float32, device="cuda")

    def step(x, meth):
        pr.step_async(rho, u, v, flags, p, x, 1e-3, g=sc.g, drho=sc.drho, u_in=sc.u_in, cfl=0.5,
                      method=meth, max_iters=200000, check_every=128 if meth == "hybrid" else 1)

    for s in range(6):  # a developed plume
        step(to_dev(scenes.inflow_noise(0, s, n)), "pcg")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step(xb, method)
    torch.cuda.synchronize()
    for s in range(6, 11):
        x = to_dev(scenes.inflow_noise(0, s, n))
        start = [t.clone() for t in (rho, u, v, p)]
        step(x, method)  # eager
        torch.cuda.synchronize()
        r_e = pr.result()
        eager = [t.clone() for t in (rho, u, v, p)]
        for d, s_ in zip((rho, u, v, p), start):
            d.copy_(s_)
        xb.copy_(x)
        g.replay()
        torch.cuda.synchronize()
        r_g = pr.result()
        say(method, "step", s, "iters", r_e.iters, r_g.iters, "status", r_e.status, r_g.status)
        assert r_g.status == r_e.status == 0 and r_g.iters == r_e.iters
        assert r_g.e1_final == r_e.e1_final and r_g.dt == r_e.dt
        assert all(torch.equal(a, b) for a, b in zip(eager, (rho, u, v, p)))
