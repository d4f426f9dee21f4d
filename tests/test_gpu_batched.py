"""Batched form: one persistent Jacobi launch over many plumes of uneven
sizes must give each instance the result of its own projection, match the
oracle at the GPU's sweep count, and replay identically from a hipGraph."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import grid as G
from oracle import project as PR
from tests.gpu_util import to_dev, f32, rel_l2, gpu_project

pytestmark = pytest.mark.gpu

SIZES = [(64, 64), (96, 64), (128, 128), (64, 160), (200, 96), (128, 72)]


def say(*a):
    print(*a, flush=True)


def make_instances(seed=0, rel=0.1):
    inst, host = [], []
    for i, (nx, ny) in enumerate(SIZES):
        sc = scenes.plume_scene(nx, seed=seed + i, n_obstacles=(0, 3), ny=ny)
        u, v = scenes.random_faces(nx, ny, seed + i, kind="mixed")
        u, v = f32(u), f32(v)
        P = G.plan(sc.flags)
        thr = rel * G.e1(P, G.divergence(P, *G.enforce_bc(P, u, v), sc.dx))
        host.append(dict(sc=sc, u=u, v=v, thr=thr))
        inst.append(dict(nx=nx, ny=ny, dx=sc.dx, flags=to_dev(sc.flags, torch.uint8), u=to_dev(u),
                         v=to_dev(v), p=torch.zeros((ny, nx), dtype=torch.float32, device="cuda"),
                         threshold=thr, dt=0.01))
    return inst, host


@pytest.mark.parametrize("check_every", [8, 64, 60])
def test_batched_jacobi_matches_single_and_oracle(check_every):
    """check_every 64: E_1 tested every 8 exchanges of 8 sweeps, the same
    sweep counts as a single projection testing every 64; 60 rounds up to
    64."""
    inst, host = make_instances()
    b = hp.Batch(inst, method="jacobi", max_iters=100000, check_every=check_every)
    b.project_async()
    torch.cuda.synchronize()
    res = b.results()
    every = -(-check_every // 8) * 8
    for i, (r, h) in enumerate(zip(res, host)):
        sc = h["sc"]
        g = gpu_project(sc.flags, h["u"], h["v"], sc.dx, thr=h["thr"], method="jacobi", dt=0.01,
                        check_every=every, max_iters=100000)
        say("inst", i, SIZES[i], "batched iters", r.iters, "single", g["res"].iters)
        assert r.status == 0
        assert r.iters % every == 0
        assert abs(r.iters - g["res"].iters) <= every
        pb = inst[i]["p"].cpu().numpy().astype(np.float64)
        o = PR.project(sc.flags, h["u"], h["v"], sc.dx, dt=0.01, method="jacobi", fixed_iters=r.iters)
        err = rel_l2(pb, o["p"], o["plan"].fluid)
        say("   rel L2 vs oracle at the same sweeps", err)
        assert err <= 1e-4
        assert r.e1_final <= 1.01 * h["thr"]


def _stepping_instances(seed, sizes=SIZES, var=False):
    """Plumes with their own physics: drho ~ U[0.01, 0.5] and g from Ri 0.1
    (Eq. 1), each from a seeded light-blob state."""
    inst, host = [], []
    rng = np.random.default_rng(seed)
    for i, (nx, ny) in enumerate(sizes):
        drho = float(rng.uniform(0.01, 0.5))
        sc = scenes.plume_scene(nx, seed=seed + i, n_obstacles=(0, 3), ny=ny, drho=drho)
        u, v = (f32(0.5 * a) for a in scenes.random_faces(nx, ny, seed + i, kind="smooth"))
        rho = f32(scenes.random_density(nx, ny, seed + i, sc.rho0, drho))
        host.append(dict(sc=sc, u=u, v=v, rho=rho))
        inst.append(dict(nx=nx, ny=ny, dx=sc.dx, flags=to_dev(sc.flags, torch.uint8), u=to_dev(u),
                         v=to_dev(v), rho=to_dev(rho), xi=torch.zeros(nx, dtype=torch.float32, device="cuda"),
                         p=torch.zeros((ny, nx), dtype=torch.float32, device="cuda"),
                         threshold=1e-1, g=sc.g, drho=drho, u_in=sc.u_in))
    return inst, host


def test_batched_hybrid_and_graph_replay():
    S, C = 3, 16
    w = scenes.random_weights(S, C, 0, out_scale=0.05)
    tw = to_dev(w)
    runs = []
    for mode in ("eager", "graph"):
        inst, host = _stepping_instances(10)
        b = hp.Batch(inst, method="hybrid", params=tw, scales=S, channels=C, max_iters=20000)
        if mode == "graph":
            b.capture()
        outs = []
        for step in range(3):
            for d in inst:
                d["xi"].copy_(torch.from_numpy(scenes.inflow_noise(1, step, d["nx"]).astype(np.float32)))
            if mode == "eager":
                b.step_async()
            else:
                b.launch_async()
            torch.cuda.synchronize()
            outs.append(([r.iters for r in b.results()], [d["u"].cpu().numpy().copy() for d in inst]))
        runs.append(outs)
        say(mode, [o[0] for o in outs])
    for (ie, ue), (ig, ug) in zip(runs[0], runs[1]):
        assert ie == ig
        for a, c in zip(ue, ug):
            assert np.array_equal(a, c)


@pytest.mark.parametrize("method", ["hybrid", "jacobi"])
def test_batched_step_equals_single_steps(method):
    """The batched time step of plumes with their own g and drho (one launch
    per phase over all of them) gives each plume exactly what its own
    hyp_step gives: same advection, network, sweeps and correction."""
    S, C = 3, 16
    w = scenes.random_weights(S, C, 3, out_scale=0.05)
    tw = to_dev(w)
    sizes = [(64, 64), (128, 96), (96, 160), (192, 192), (64, 128)]
    inst, host = _stepping_instances(30, sizes)
    kw = dict(params=tw, scales=S, channels=C) if method == "hybrid" else {}
    b = hp.Batch(inst, method=method, max_iters=20000, **kw)
    for d in inst:
        d["xi"].copy_(torch.from_numpy(scenes.inflow_noise(2, 0, d["nx"]).astype(np.float32)))
    b.step_async()
    torch.cuda.synchronize()
    res = b.results()
    for i, (d, h) in enumerate(zip(inst, host)):
        sc = h["sc"]
        pr = hp.Projector(d["nx"], d["ny"], sc.dx, 1.0, sc.rho0, S if method == "hybrid" else 0, C, "fp32")
        if method == "hybrid":
            pr.set_weights(tw)
        tf = to_dev(sc.flags, torch.uint8)
        pr.plan(tf)
        rho, u, v = to_dev(h["rho"]), to_dev(h["u"]), to_dev(h["v"])
        p = torch.zeros((d["ny"], d["nx"]), dtype=torch.float32, device="cuda")
        # no defect-correction folds on the single grid (the batch has none),
        # so that both take the same FP32 path
        pr.step_async(rho, u, v, tf, p, d["xi"].clone(), 1e-1, g=d["g"], drho=d["drho"], u_in=d["u_in"],
                      method=method, check_every=8, max_iters=20000, fold_window=1 << 30)
        torch.cuda.synchronize()
        r = pr.result()
        say("inst", i, sizes[i], "drho", round(d["drho"], 3), "batched", res[i].iters, res[i].dt,
            "single", r.iters, r.dt)
        assert res[i].status in (0, 1) and res[i].status == r.status
        assert res[i].dt == r.dt and res[i].iters == r.iters
        for a, c in ((d["rho"], rho), (d["u"], u), (d["v"], v), (d["p"], p)):
            an, cn = a.cpu().numpy(), c.cpu().numpy()
            assert np.abs(an - cn).max() <= 1e-6 * max(np.abs(cn).max(), 1e-30)


def test_batched_variable_density_matches_oracle():
    """Variable density in the batch (each plume its own density field, up
    to half the reference density): each instance's pressure matches the
    oracle's variable-coefficient Jacobi at the batch's sweep count, and its
    count the single-grid variable-density kernel's within one test."""
    from oracle import varcoef as VC
    from tests.gpu_util import gpu_project
    sizes = [(64, 64), (128, 96), (96, 160), (192, 192)]
    inst, host = _stepping_instances(50, sizes)
    for d, h in zip(inst, host):
        P = G.plan(h["sc"].flags)
        d["threshold"] = 0.2 * G.e1(P, G.divergence(P, *G.enforce_bc(P, h["u"], h["v"]), h["sc"].dx))
    b = hp.Batch(inst, method="jacobi", max_iters=200000, variable_density=True)
    b.project_async()
    torch.cuda.synchronize()
    res = b.results()
    for i, (d, h) in enumerate(zip(inst, host)):
        sc = h["sc"]
        P = G.plan(sc.flags)
        ub, vb = G.enforce_bc(P, h["u"], h["v"])
        dd = G.divergence(P, ub, vb, sc.dx)
        bu, bv = VC.face_coefficients(P, h["rho"], sc.rho0)
        phi, k, st = VC.jacobi(P, dd, bu, bv, sc.dx, fixed_iters=res[i].iters)
        pb = d["p"].cpu().numpy().astype(np.float64)
        err = rel_l2(pb, sc.rho0 * phi / 1.0, P.fluid)
        g = gpu_project(sc.flags, h["u"], h["v"], sc.dx, thr=d["threshold"], method="jacobi", check_every=8,
                        max_iters=200000, rho=to_dev(h["rho"]), variable_density=True)
        say("inst", i, sizes[i], "iters", res[i].iters, g["res"].iters, "rel L2 p", err)
        assert res[i].status == 0 and abs(res[i].iters - g["res"].iters) <= 8
        assert err <= 1e-4


def _instances(sizes, seed, thr):
    inst, host = [], []
    for i, (nx, ny) in enumerate(sizes):
        sc = scenes.plume_scene(nx, seed=seed + i, n_obstacles=(0, 3), ny=ny)
        u, v = scenes.random_faces(nx, ny, seed + i, kind="mixed")
        u, v = f32(u), f32(v)
        P = G.plan(sc.flags)
        t = thr if thr is not None else 0.2 * G.e1(P, G.divergence(P, *G.enforce_bc(P, u, v), sc.dx))
        host.append(dict(sc=sc, u=u, v=v, thr=t))
        inst.append(dict(nx=nx, ny=ny, dx=sc.dx, flags=to_dev(sc.flags, torch.uint8), u=to_dev(u),
                         v=to_dev(v), p=torch.zeros((ny, nx), dtype=torch.float32, device="cuda"),
                         threshold=t, dt=0.01))
    return inst, host


def test_batched_fixed_sweeps_many_tiles_per_workgroup():
    """More tiles than resident work-groups (one 2048^2 grid is 2,025 tiles
    of the batched kernel, plus 16 plumes with sides from {128, ..., 512}),
    so every work-group sweeps several tiles per pass; threshold 0 runs
    every instance for exactly max_iters sweeps, and each must match the
    oracle's Jacobi at that count."""
    rng = np.random.default_rng(5)
    sides = [128, 192, 256, 384, 512]
    sizes = [(2048, 2048)] + [(int(s), int(s)) for s in rng.choice(sides, 16)]
    k = 96
    inst, host = _instances(sizes, 40, thr=0.0)
    b = hp.Batch(inst, method="jacobi", max_iters=k)
    b.project_async()
    torch.cuda.synchronize()
    res = b.results()
    for i, (r, h) in enumerate(zip(res, host)):
        sc = h["sc"]
        assert r.status == 1 and r.iters == k  # MAXITER: the fixed count
        pb = inst[i]["p"].cpu().numpy().astype(np.float64)
        o = PR.project(sc.flags, h["u"], h["v"], sc.dx, dt=0.01, method="jacobi", fixed_iters=k)
        err = rel_l2(pb, o["p"], o["plan"].fluid)
        eu = rel_l2(inst[i]["u"].cpu().numpy().astype(np.float64), o["u"])
        say("inst", i, sizes[i], "rel L2 p", err, "u", eu)
        assert err <= 1e-4 and eu <= 1e-5


def test_batched_threshold_cfg4_style_draw():
    """A draw of 20 plumes with sides from {128, ..., 512} and 0-3 disks
    projected together to 20 % of each one's initial E_1: every instance's
    sweep count is the single-grid kernel's within one test interval, and
    its pressure the oracle's at that count."""
    rng = np.random.default_rng(6)
    sides = [128, 192, 256, 384, 512]
    sizes = [(int(s), int(s)) for s in rng.choice(sides, 20)]
    inst, host = _instances(sizes, 70, thr=None)
    b = hp.Batch(inst, method="jacobi", max_iters=200000)
    b.project_async()
    torch.cuda.synchronize()
    res = b.results()
    for i, (r, h) in enumerate(zip(res, host)):
        sc = h["sc"]
        g = gpu_project(sc.flags, h["u"], h["v"], sc.dx, thr=h["thr"], method="jacobi", dt=0.01,
                        check_every=8, max_iters=200000)
        assert r.status == 0 and abs(r.iters - g["res"].iters) <= 8
        pb = inst[i]["p"].cpu().numpy().astype(np.float64)
        o = PR.project(sc.flags, h["u"], h["v"], sc.dx, dt=0.01, method="jacobi", fixed_iters=r.iters)
        err = rel_l2(pb, o["p"], o["plan"].fluid)
        say("inst", i, sizes[i], "iters", r.iters, g["res"].iters, "rel L2 p", err)
        assert err <= 1e-4
        assert r.e1_final <= 1.01 * h["thr"]
