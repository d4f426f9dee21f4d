"""Measurements beside the headline benchmark (one JSON object per line).

python -m paper_2109_09363_amd.experiments WHAT [options]

WHAT:
  thresholds  512^2 plumes (seeds 0-4, 0-3 disks): after `warmup` PCG-projected
              steps, `steps` time steps from the same state with the hybrid
              (4-scale 64-channel BF16 net, and the same weights in FP32) and
              with PCG, for each threshold 1e-2, 1e-3, 1e-4; sweeps/iterations
              per step, ms per step, statuses, and the BF16-vs-FP32 distance
              of the CNN guess and of the returned pressure.
  gain        the same 512^2 states: trained net vs zero net (= plain
              Jacobi) vs seeded random net vs PCG, at 1e-3.
  batch       128 plumes, sides from {128, 192, 256, 384, 512}, 0-3 disks,
              density ratio ~ U[0.01, 0.5] (seed 0): one batched step (per
              instance advection, divergence, CNN, then one persistent
              Jacobi launch for all instances) to 1e-3, eager and as a
              captured graph; per-instance sweeps.
  dram        the streaming (batched) Jacobi kernel on one large grid
              (default 8192^2, 268 MB per FP32 field) for a fixed number of
              sweeps: algorithmic bytes per second against the HBM peak.
  validate    model selection for network weights: 512^2 plumes of --seeds
              (default 100-107, disjoint from the benchmark's seed 0, the
              experiments' seeds 0-4 and the training scenes), each developed
              by `warmup` PCG steps, then `steps` hybrid steps to 1e-3 with
              every candidate in --weights from the same state; mean sweeps
              and ms per step per candidate.
  checks      hybrid ms per step against the E_1 test interval (validation
              plumes, --intervals).
  networks    inference time t_inf (divergence + network, the library's phase
              events) of every network on grids of --sizes (default 512):
              the parallel 4-scale 64-channel and 3-scale 32-channel nets and
              the paper's cascaded MultiScale and SmallScale and its Unet,
              FP32 and BF16;
              MFMA FLOP/s against the dense peaks (Sec. 5.1, Table 1).
All inputs are seeded and synthetic; timings use the stream's HIP events
(through torch.cuda.Event on the current stream, which the library uses).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenes  # noqa: E402
import paper_2109_09363_amd as hp  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "plume_s4c64.npy")
S4, C64 = 4, 64


def emit(obj):
    print(json.dumps(obj), flush=True)


class Plume:
    """One 512^2 plume developed by PCG-projected steps; snapshot/restore."""

    def __init__(self, n, seed, warmup, dev, weights, precision="bf16"):
        self.sc = scenes.plume_scene(n, seed=seed, n_obstacles=(0, 3))
        self.n, self.seed = n, seed
        self.flags = torch.from_numpy(self.sc.flags).to(dev)
        self.pr = hp.Projector(n, n, self.sc.dx, 1.0, self.sc.rho0, S4, C64, precision, device=dev)
        self.pr.set_weights(weights)
        self.pr.plan(self.flags)
        self.rho = torch.full((n, n), self.sc.rho0, dtype=torch.float32, device=dev)
        self.u = torch.zeros((n, n + 1), dtype=torch.float32, device=dev)
        self.v = torch.zeros((n + 1, n), dtype=torch.float32, device=dev)
        self.p = torch.zeros((n, n), dtype=torch.float32, device=dev)
        self.xi = [torch.from_numpy(scenes.inflow_noise(seed, s, n).astype(np.float32)).to(dev)
                   for s in range(warmup + 400)]
        self.warmup = warmup
        for s in range(warmup):
            self.step("pcg", 1e-3, s)
        torch.cuda.synchronize()
        self.snap = [t.clone() for t in (self.rho, self.u, self.v, self.p)]

    def restore(self):
        for dst, src in zip((self.rho, self.u, self.v, self.p), self.snap):
            dst.copy_(src)
        torch.cuda.synchronize()

    check_every = 8  # E_1 test interval of the hybrid (PCG tests every iteration)

    def step(self, method, thr, s, pr=None):
        ce = self.check_every if method != "pcg" else 1
        (pr or self.pr).step_async(self.rho, self.u, self.v, self.flags, self.p, self.xi[s], thr,
                                   g=self.sc.g, drho=self.sc.drho, u_in=self.sc.u_in, cfl=0.5,
                                   method=method, max_iters=1000000, check_every=ce)

    def run(self, method, thr, steps, pr=None):
        """`steps` time steps from the snapshot; per-step results and the
        event-timed total.  The first step's pressure is kept in first_p."""
        self.restore()
        pr = pr or self.pr
        rows = []
        t_ms = 0.0
        for s in range(self.warmup, self.warmup + steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            self.step(method, thr, s, pr)
            b.record()
            torch.cuda.synchronize()
            t_ms += a.elapsed_time(b)
            rows.append(pr.result())
            if s == self.warmup:
                self.first_p = self.p.cpu().numpy().copy()
                self.first_dt = rows[-1].dt
        return rows, t_ms

    def first_inputs(self):
        """What the first timed step's projection receives: the snapshot
        advected once (deterministic, the same for every method), with that
        step's dt."""
        self.restore()
        rho, u, v = self.rho.clone(), self.u.clone(), self.v.clone()
        self.pr.advect_async(rho, u, v, self.xi[self.warmup], g=self.sc.g, drho=self.sc.drho,
                             u_in=self.sc.u_in, cfl=0.5)
        torch.cuda.synchronize()
        return dict(flags=self.sc.flags, u=u.cpu().numpy(), v=v.cpu().numpy(), dx=self.sc.dx,
                    dt=self.first_dt, rho0=self.sc.rho0)


class Saver:
    """--save DIR: per plume, the first timed step's projection inputs and
    every method's returned pressure for that step (float32 .npz), so that
    the errors against the FP64 oracle can be computed afterwards by a
    separate process (the library never runs the oracle)."""

    def __init__(self, root, what):
        self.dir = os.path.join(root, what) if root else None
        if self.dir:
            os.makedirs(self.dir, exist_ok=True)

    def save(self, name, inputs, cases):
        if not self.dir:
            return
        arrays = {"flags": inputs["flags"], "u": inputs["u"], "v": inputs["v"],
                  "scalars": np.array([inputs["dx"], inputs["dt"], inputs["rho0"]])}
        meta = []
        for i, c in enumerate(cases):
            arrays[f"p{i}"] = c.pop("p").astype(np.float32)
            meta.append(c)
        np.savez(os.path.join(self.dir, name + ".npz"), **arrays)
        with open(os.path.join(self.dir, name + ".json"), "w") as f:
            json.dump(meta, f)


def summarize(rows, t_ms, steps):
    it = np.array([r.iters for r in rows], dtype=np.float64)
    return {"timesteps_per_s": round(steps / (t_ms * 1e-3), 3), "ms_per_step": round(t_ms / steps, 4),
            "mean_iters": round(float(it.mean()), 1), "max_iters": int(it.max()),
            "statuses": sorted(set(int(r.status) for r in rows)),
            "max_e1_final": max(r.e1_final for r in rows)}


def load_trained(dev):
    w = np.load(WEIGHTS, allow_pickle=False).astype(np.float32)
    return torch.from_numpy(w).to(dev)


def cmd_thresholds(a, dev):
    w = load_trained(dev)
    saver = Saver(a.save, "thresholds")
    for seed in a.seeds:
        pl = Plume(512, seed, a.warmup, dev, w)
        cases = []
        pr32 = hp.Projector(512, 512, pl.sc.dx, 1.0, pl.sc.rho0, S4, C64, "fp32", device=dev)
        pr32.set_weights(w)
        pr32.plan(pl.flags)
        # BF16 vs FP32 network on the snapshot's advected state (guess only)
        pl.restore()
        pl.pr.advect_async(pl.rho, pl.u, pl.v, pl.xi[pl.warmup], g=pl.sc.g, drho=pl.sc.drho)
        u0, v0 = pl.u.clone(), pl.v.clone()
        guesses = []
        for pr in (pl.pr, pr32):
            uu, vv = u0.clone(), v0.clone()
            p = torch.zeros_like(pl.p)
            pr.project_async(uu, vv, pl.flags, p, 0.0, method="cnn")
            torch.cuda.synchronize()
            guesses.append(p.clone())
        d_guess = float(torch.linalg.norm(guesses[0] - guesses[1]) / torch.linalg.norm(guesses[1]))
        for thr in a.thresholds:
            out = {"what": "thresholds", "seed": seed, "threshold": thr, "n_obstacles": len(pl.sc.disks),
                   "steps": a.steps, "cnn_guess_bf16_vs_fp32_rel_l2": d_guess}
            rows, t = pl.run("hybrid", thr, a.steps)
            out["hybrid_bf16"] = summarize(rows, t, a.steps)
            cases.append(dict(method="hybrid", precision="bf16", threshold=thr, iters=int(rows[0].iters),
                              check_every=pl.check_every, p=pl.first_p))
            p_bf = pl.p.clone()
            rows, t = pl.run("hybrid", thr, a.steps, pr32)
            out["hybrid_fp32"] = summarize(rows, t, a.steps)
            cases.append(dict(method="hybrid", precision="fp32", threshold=thr, iters=int(rows[0].iters),
                              check_every=pl.check_every, p=pl.first_p))
            out["final_p_bf16_vs_fp32_rel_l2"] = float(torch.linalg.norm(p_bf - pl.p) / torch.linalg.norm(pl.p))
            rows, t = pl.run("pcg", thr, a.steps)
            out["pcg"] = summarize(rows, t, a.steps)
            cases.append(dict(method="pcg", precision="fp32", threshold=thr, iters=int(rows[0].iters),
                              check_every=1, p=pl.first_p))
            out["hybrid_over_pcg"] = round(out["pcg"]["ms_per_step"] / out["hybrid_bf16"]["ms_per_step"], 4)
            emit(out)
        saver.save(f"seed{seed}", pl.first_inputs(), cases)


def cmd_gain(a, dev):
    nets = {"trained": load_trained(dev),
            "zero": torch.zeros(scenes.cnn_param_count(S4, C64), dtype=torch.float32, device=dev),
            "random": torch.from_numpy(scenes.random_weights(S4, C64, 7).astype(np.float32)).to(dev)}
    saver = Saver(a.save, "gain")
    for seed in a.seeds:
        pl = Plume(512, seed, a.warmup, dev, nets["trained"])
        out = {"what": "gain", "seed": seed, "threshold": 1e-3, "steps": a.steps, "n_obstacles": len(pl.sc.disks)}
        cases = []
        for name, w in nets.items():
            pl.pr.set_weights(w)
            rows, t = pl.run("hybrid", 1e-3, a.steps)
            out["hybrid_" + name] = summarize(rows, t, a.steps)
            cases.append(dict(method="hybrid", precision="bf16", weights=name, threshold=1e-3,
                              iters=int(rows[0].iters), check_every=pl.check_every, p=pl.first_p))
        pl.pr.set_weights(nets["trained"])
        rows, t = pl.run("pcg", 1e-3, a.steps)
        out["pcg"] = summarize(rows, t, a.steps)
        cases.append(dict(method="pcg", precision="fp32", threshold=1e-3, iters=int(rows[0].iters),
                          check_every=1, p=pl.first_p))
        emit(out)
        saver.save(f"seed{seed}", pl.first_inputs(), cases)


def batch_instances(dev, n_inst=128, seed=0):
    rng = np.random.default_rng(seed)
    sides = [128, 192, 256, 384, 512]
    inst = []
    for i in range(n_inst):
        s = int(rng.choice(sides))
        drho = float(rng.uniform(0.01, 0.5))
        sc = scenes.plume_scene(s, seed=1000 + i, n_obstacles=(0, 3), drho=drho)
        inst.append(dict(nx=s, ny=s, dx=sc.dx, dt=1.0, rho0=sc.rho0, scene=sc,
                         flags=torch.from_numpy(sc.flags).to(dev),
                         rho=torch.full((s, s), sc.rho0, dtype=torch.float32, device=dev),
                         u=torch.zeros((s, s + 1), dtype=torch.float32, device=dev),
                         v=torch.zeros((s + 1, s), dtype=torch.float32, device=dev),
                         p=torch.zeros((s, s), dtype=torch.float32, device=dev),
                         xi=torch.from_numpy(scenes.inflow_noise(1000 + i, 0, s).astype(np.float32)).to(dev)))
    return inst


def cmd_batch(a, dev):
    """The batched workload: 128 plumes with their own sides, obstacles and
    density ratios (so their own g), developed by PCG-projected steps, then
    one projection of all of them and batched time steps (each plume its own
    physics) replayed from one captured hipGraph."""
    inst = batch_instances(dev)
    cells = sum(d["nx"] * d["ny"] for d in inst)
    w = load_trained(dev)
    for d in inst:
        sc = d["scene"]
        d["g"], d["drho"], d["u_in"] = sc.g, sc.drho, sc.u_in
        pr = hp.Projector(d["nx"], d["ny"], sc.dx, 1.0, sc.rho0, S4, C64, "bf16", device=dev)
        pr.set_weights(w)
        pr.plan(d["flags"])
        for s in range(a.warmup):
            xi = torch.from_numpy(scenes.inflow_noise(1000, s, d["nx"]).astype(np.float32)).to(dev)
            pr.step_async(d["rho"], d["u"], d["v"], d["flags"], d["p"], xi, 1e-3, g=sc.g, drho=sc.drho,
                          method="pcg", max_iters=200000)
        d["_pr"] = pr
    torch.cuda.synchronize()
    # developed (projected) states, the start of the timed steps
    snap_step = [(d["rho"].clone(), d["u"].clone(), d["v"].clone(), d["p"].clone()) for d in inst]
    # and their next advected states, what the timed projections receive
    for d in inst:
        sc = d["scene"]
        xi = torch.from_numpy(scenes.inflow_noise(1000, a.warmup, d["nx"]).astype(np.float32)).to(dev)
        d.pop("_pr").advect_async(d["rho"], d["u"], d["v"], xi, g=sc.g, drho=sc.drho)
    torch.cuda.synchronize()
    snap_proj = [(d["rho"].clone(), d["u"].clone(), d["v"].clone(), d["p"].clone()) for d in inst]

    def restore(snap):
        for d, (r, u, v, p) in zip(inst, snap):
            d["rho"].copy_(r); d["u"].copy_(u); d["v"].copy_(v); d["p"].copy_(p)
        torch.cuda.synchronize()

    def timed(fn, reps, snap):
        ts = []
        for _ in range(reps):
            restore(snap)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return float(np.median(ts))

    out = {"what": "batch", "instances": len(inst), "cells": cells, "threshold": 1e-3,
           "sides": sorted(set(d["nx"] for d in inst)), "variable_density": bool(a.var),
           "check_every": a.check_every}
    saver = Saver(a.save, "batch")
    sample = list(range(0, len(inst), 8))  # the instances whose results are saved
    cases = {i: [] for i in sample}
    for method in ("hybrid", "jacobi"):
        b = hp.Batch(inst, threshold=1e-3, method=method, params=w, scales=S4, channels=C64,
                     precision="bf16", max_iters=400000, variable_density=bool(a.var),
                     check_every=a.check_every)
        restore(snap_proj)
        b.project_async()          # warm
        torch.cuda.synchronize()
        ms_proj = timed(b.project_async, 3, snap_proj)
        res = b.results()
        for i in sample:
            cases[i].append(dict(method=method, precision="bf16", weights="trained" if method == "hybrid"
                                 else "none", threshold=1e-3, iters=int(res[i].iters),
                                 check_every=a.check_every,
                                 variable_density=bool(a.var), p=inst[i]["p"].cpu().numpy().copy()))
        it = np.array([r.iters for r in res], dtype=np.float64)
        row = {"ms_per_projection_of_all": round(ms_proj, 3),
               "mean_sweeps": round(float(it.mean()), 1), "max_sweeps": int(it.max()),
               "min_sweeps": int(it.min()), "statuses": sorted(set(int(r.status) for r in res)),
               "max_e1_final": max(r.e1_final for r in res)}
        if method == "hybrid":
            # batched time steps, each plume with its own g, drho and dt
            ms_eager = timed(b.step_async, 3, snap_step)
            b.capture()
            ms_graph = timed(b.launch_async, 3, snap_step)
            res = b.results()
            row.update({"ms_per_step_of_all_eager": round(ms_eager, 3),
                        "ms_per_step_of_all_graph": round(ms_graph, 3),
                        "timesteps_per_s_per_plume_graph": round(1e3 / ms_graph, 2),
                        "step_statuses": sorted(set(int(r.status) for r in res)),
                        "step_mean_sweeps": round(float(np.mean([r.iters for r in res])), 1)})
        out[method] = row
        del b
    emit(out)
    for i in sample:
        d, (r, u, v, _p) = inst[i], snap_proj[i]
        saver.save(f"inst{i:03d}", dict(flags=d["scene"].flags, u=u.cpu().numpy(), v=v.cpu().numpy(),
                                        dx=d["dx"], dt=d["dt"], rho0=d["rho0"]), cases[i])
        if saver.dir:
            np.save(os.path.join(saver.dir, f"inst{i:03d}_rho.npy"), r.cpu().numpy())


def cmd_dram(a, dev):
    n = a.n
    sc = scenes.plume_scene(n, seed=0, n_obstacles=2)
    u, v = scenes.random_faces(n, n, 0, kind="white")
    inst = [dict(nx=n, ny=n, dx=sc.dx, flags=torch.from_numpy(sc.flags).to(dev),
                 u=torch.from_numpy(u.astype(np.float32)).to(dev),
                 v=torch.from_numpy(v.astype(np.float32)).to(dev),
                 p=torch.zeros((n, n), dtype=torch.float32, device=dev))]
    b = hp.Batch(inst, threshold=0.0, method="jacobi", max_iters=a.sweeps, check_every=a.check_every)
    b.project_async()
    torch.cuda.synchronize()
    times = []
    for _ in range(a.reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.project_async()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    r = b.results()[0]
    ms = float(np.median(times))
    algo = 13.0 * n * n * r.iters
    emit({"what": "dram", "n": n, "sweeps": int(r.iters), "status": int(r.status),
          "check_every": a.check_every,
          "ms_per_projection": round(ms, 3), "us_per_sweep": round(1e3 * ms / max(r.iters, 1), 3),
          "algorithmic_GBps": round(algo / (ms * 1e-3) / 1e9, 1), "hbm_peak_GBps": 8000.0,
          "note": "the projection also runs the divergence, gradient and check passes"})


def cmd_checks(a, dev):
    """Hybrid ms per step against the E_1 test interval on the validation
    plumes (a test costs about one sweep; a long interval overshoots)."""
    w = load_trained(dev)
    res = {ce: [0.0, 0.0] for ce in a.intervals}
    for seed in a.seeds:
        pl = Plume(512, seed, a.warmup, dev, w)
        for ce in a.intervals:
            pl.check_every = ce
            rows, t = pl.run("hybrid", 1e-3, a.steps)
            sm = summarize(rows, t, a.steps)
            res[ce][0] += sm["ms_per_step"] / len(a.seeds)
            res[ce][1] += sm["mean_iters"] / len(a.seeds)
    emit({"what": "checks", "seeds": a.seeds, "steps": a.steps,
          "ms_per_step": {ce: round(v[0], 4) for ce, v in res.items()},
          "mean_sweeps": {ce: round(v[1], 1) for ce, v in res.items()}})


def cmd_validate(a, dev):
    cands = {os.path.basename(f): torch.from_numpy(np.load(f, allow_pickle=False).astype(np.float32)).to(dev)
             for f in a.weights}
    first = next(iter(cands.values()))
    tot = {k: [0.0, 0.0] for k in cands}
    for seed in a.seeds:
        pl = Plume(512, seed, a.warmup, dev, first)
        out = {"what": "validate", "seed": seed, "steps": a.steps, "n_obstacles": len(pl.sc.disks)}
        for name, w in cands.items():
            pl.pr.set_weights(w)
            rows, t = pl.run("hybrid", 1e-3, a.steps)
            sm = summarize(rows, t, a.steps)
            out[name] = {"mean_sweeps": sm["mean_iters"], "ms_per_step": sm["ms_per_step"]}
            tot[name][0] += sm["mean_iters"] / len(a.seeds)
            tot[name][1] += sm["ms_per_step"] / len(a.seeds)
        emit(out)
    emit({"what": "validate", "seeds": a.seeds,
          "mean": {k: {"mean_sweeps": round(v[0], 1), "ms_per_step": round(v[1], 4)} for k, v in tot.items()}})


# network configurations: (label, arch, scales, channels)
NETWORKS = [("parallel S4 C64", "parallel", 4, 64), ("parallel S3 C32", "parallel", 3, 32),
            ("MultiScale", "multiscale", 3, 64), ("SmallScale", "smallscale", 3, 32),
            ("Unet", "unet", 5, 64)]
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}


def net_macs(arch, scales, channels, nx, ny):
    """Multiply-adds of one inference (every convolution, all scales)."""
    if arch == "parallel":
        C = channels
        per_px = 9 * 2 * C + 3 * 9 * C * C + C
        return sum(per_px * (nx >> k) * (ny >> k) for k in range(scales))
    if arch == "unet":
        layers = scenes.paper_net_layers("unet")[0]
        levels = [l for l in range(5) for _ in range(2)] + [l for l in range(3, -1, -1) for _ in range(2)]
        levels.append(0)
        return sum(k * k * ci * co * (nx >> lv) * (ny >> lv) for (k, ci, co), lv in zip(layers, levels))
    total = 0
    for b, br in enumerate(scenes.paper_net_layers(arch)):
        f = 4 >> b
        total += sum(k * k * ci * co for (k, ci, co) in br) * (nx // f) * (ny // f)
    return total


def cmd_networks(a, dev):
    for n in a.sizes:
        sc = scenes.plume_scene(n, seed=0, n_obstacles=2)
        u, v = scenes.random_faces(n, n, 0, kind="mixed")
        flags = torch.from_numpy(sc.flags).to(dev)
        u0 = torch.from_numpy(u.astype(np.float32)).to(dev)
        v0 = torch.from_numpy(v.astype(np.float32)).to(dev)
        p = torch.empty((n, n), dtype=torch.float32, device=dev)
        for (label, arch, S, C) in NETWORKS:
            for prec in ("fp32", "bf16"):
                if arch == "parallel" and prec == "bf16" and C == 16:
                    continue
                pr = hp.Projector(n, n, sc.dx, 1.0, 1.0, S, C, prec, device=dev, arch=arch)
                if arch == "parallel":
                    w = scenes.random_weights(S, C, 0)
                else:
                    w = scenes.random_paper_weights(arch, 0)
                tw = torch.from_numpy(w).to(dev)
                pr.set_weights(tw)
                pr.plan(flags)
                pr.set_timing(True)
                ts = []
                for rep in range(a.reps + 3):
                    uu, vv = u0.clone(), v0.clone()
                    pr.project_async(uu, vv, flags, p, 0.0, method="cnn")
                    torch.cuda.synchronize()
                    if rep >= 3:
                        ts.append(pr.timing()["inference"])
                ms = float(np.median(ts))
                macs = net_macs(arch, S, C, n, n)
                tf = 2.0 * macs / (ms * 1e-3) / 1e12
                emit({"what": "networks", "n": n, "net": label, "params": int(w.size),
                      "precision": prec, "t_inf_ms": round(ms, 4), "gflop": round(2 * macs / 1e9, 2),
                      "tflops": round(tf, 1), "mfma_peak_tflops": PEAK_TFLOPS[prec],
                      "frac_of_peak": round(tf / PEAK_TFLOPS[prec], 4)})
                del pr


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["thresholds", "gain", "batch", "dram", "networks", "validate",
                                     "checks"])
    ap.add_argument("--intervals", type=int, nargs="*", default=[8, 16, 32, 64, 128])
    ap.add_argument("--weights", nargs="*", default=[WEIGHTS])
    ap.add_argument("--sizes", type=int, nargs="*", default=[512])
    ap.add_argument("--seeds", type=int, nargs="*", default=None)
    ap.add_argument("--thresholds", type=float, nargs="*", default=[1e-2, 1e-3, 1e-4])
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--n", type=int, default=8192)
    ap.add_argument("--sweeps", type=int, default=800)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--var", action="store_true", help="batch: variable-density operator")
    ap.add_argument("--check-every", type=int, default=None,
                    help="batch, dram: E_1 test interval in sweeps, rounded up to whole exchanges of 8 "
                         "(default: batch 64, dram only at the end)")
    ap.add_argument("--save", default=None,
                    help="thresholds, gain, batch: write the first step's projection inputs and "
                         "pressures under this folder (for the error against the FP64 oracle)")
    a = ap.parse_args()
    if a.check_every is None:
        a.check_every = a.sweeps if a.what == "dram" else 64
    if a.seeds is None:
        a.seeds = list(range(100, 108)) if a.what in ("validate", "checks") else [0, 1, 2, 3, 4]
    dev = torch.device("cuda")
    t0 = time.time()
    {"thresholds": cmd_thresholds, "gain": cmd_gain, "batch": cmd_batch, "dram": cmd_dram,
     "networks": cmd_networks, "validate": cmd_validate, "checks": cmd_checks}[a.what](a, dev)
    print(f"# {a.what} done in {time.time() - t0:.1f} s", file=sys.stderr, flush=True)


if __name__ == "__main__":
    main()
