#!/usr/bin/env python3
"""Benchmark: time steps per second of the 512x512 plume with the hybrid
CNN + Jacobi projection to mean|div u| < 1e-3, against plain FP32 PCG on
the same GPU, with the roofline of the dominant kernel and the CPU oracle
timed beside it.

python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: 512x512 unit-square plume (walls left/right/bottom, open top,
inflow width 0.16, drho 0.01, Ri 0.1), 0-3 random disks drawn from seed 0;
4-scale 64-channel BF16 CNN (FP32 accumulation, FP32 output layer) and FP32
Jacobi (omega 1, E_1 tested every 768 sweeps).  The plume is first developed for
`warmup` untimed steps projected by PCG (every step converged), then `steps`
hybrid steps are timed from that state; the same `steps` are then replayed
from the same state with PCG.  All inputs are seeded and synthetic.  On
the host the FP64 oracle then replays the first timed step (timed: the
cpu_baseline) and the GPU's pressures are compared with the oracle's on the
same inputs (error_vs_fp64_oracle).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 512
SCALES, CHANNELS = 4, 64
THRESHOLD = 1e-3
# E_1 test interval: the hybrid's test (residual, grid reduction and its
# round trip) costs several sweeps' time against the steps between tests,
# which exchange tagged halo words only, so at ~3,000-4,000 sweeps per step a
# test every 768 sweeps minimises test cost plus overshoot (measured on
# held-out plumes: experiments checks); PCG's merged reduction carries E_1
# every iteration at no extra cost
CHECK_EVERY = {"hybrid": 768, "pcg": 1}
MAX_ITERS = 1000000
BYTES_PER_CELL_SWEEP = 13   # phi read + write (8), d (4), flags (1)
HBM_PEAK_GBS = 8000.0
WEIGHTS = os.path.join(ROOT, "paper_2109_09363_amd", "weights", "plume_s4c64.npy")
# HBM traffic of the Jacobi kernel per dispatch of this benchmark, from two
# rocprofv3 counter passes (FETCH_SIZE, WRITE_SIZE) scaled by a copy kernel's
# reading; used only while the kernel's sources are unchanged since then
TRAFFIC = os.path.join(ROOT, "profiles", "jacobi_reg_plume512_traffic.txt")


def measured_traffic():
    from paper_2109_09363_amd import profsummary as PS
    if not os.path.exists(TRAFFIC):
        return None, "no counter summary"
    t = PS.read_traffic(TRAFFIC)
    if t.get("source_sha") != PS.source_hash("jacobi_reg"):
        return None, "kernel changed since the counters were taken"
    return float(t["traffic_bytes_per_dispatch"]), os.path.relpath(TRAFFIC, ROOT)


def load_weights(scenes):
    if os.path.exists(WEIGHTS):
        w = np.load(WEIGHTS, allow_pickle=False).astype(np.float32)
        if w.size == scenes.cnn_param_count(SCALES, CHANNELS):
            return w, "trained (solver-in-the-loop, " + os.path.basename(WEIGHTS) + ")"
    # untrained: random hidden layers, zero output layer (prediction = 0)
    w = scenes.random_weights(SCALES, CHANNELS, seed=0, out_scale=0.0)
    return w, "untrained (seeded random hidden layers, zero output layer)"


def oracle_leg(sc, flags, pre, ustar, gpu, w_np):
    """The FP64 oracle on the host, on the first timed step: (1) one full
    oracle time step, timed (its advection from the GPU's pre-step state,
    then the same-algorithm hybrid replica, BF16-emulated network and the
    GPU's sweep count, on the GPU's advected faces), which is the
    cpu_baseline; (2) the error of the GPU's results against the oracle's on
    the same inputs: the hybrid's pressure against that replica and against
    the replica with the unemulated FP64 network, and both methods'
    pressures against the exact FP64 solve."""
    from oracle import advect as AD, grid as G, project as PR, solve as SV
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = os.cpu_count() or 1
    P = G.plan(flags)
    rho0_, u0_, v0_, xi = pre
    us, vs = ustar
    dt = gpu["dt"]
    t0 = time.perf_counter()
    AD.advect_step(P, flags, rho0_, u0_, v0_, sc.dx, dt, sc.g, sc.rho0, sc.drho, sc.u_in, xi)
    t_adv = time.perf_counter() - t0
    k = gpu["hybrid_iters"]
    t0 = time.perf_counter()
    o = PR.project(flags, us, vs, sc.dx, dt=dt, rho0=sc.rho0, method="hybrid", params=w_np, S=SCALES,
                   C=CHANNELS, bf16=True, fixed_iters=k) if k > 0 else \
        PR.project(flags, us, vs, sc.dx, dt=dt, rho0=sc.rho0, method="cnn", params=w_np, S=SCALES,
                   C=CHANNELS, bf16=True)
    t_proj = time.perf_counter() - t0
    t0 = time.perf_counter()
    o_pcg = PR.project(flags, us, vs, sc.dx, dt=dt, rho0=sc.rho0, method="pcg", threshold=THRESHOLD,
                       check_every=1)
    t_pcg = time.perf_counter() - t0
    o64 = PR.project(flags, us, vs, sc.dx, dt=dt, rho0=sc.rho0, method="hybrid", params=w_np, S=SCALES,
                     C=CHANNELS, bf16=False, fixed_iters=k) if k > 0 else o
    ub, vb = G.enforce_bc(P, us, vs)
    ex = sc.rho0 / dt * SV.exact_solve(P, G.divergence(P, ub, vb, sc.dx), sc.dx)

    def rel(a, b):
        return float(np.linalg.norm((a - b)[P.fluid]) / max(np.linalg.norm(b[P.fluid]), 1e-300))

    def rel_uv(p_a):
        # the velocity a pressure leaves (Eq. 2) against the exactly projected one
        ue, ve = G.correct(P, ub, vb, ex * dt / sc.rho0, sc.dx)
        ua, va = G.correct(P, ub, vb, p_a * dt / sc.rho0, sc.dx)
        return float(np.sqrt((np.sum((ua - ue) ** 2) + np.sum((va - ve) ** 2))
                             / (np.sum(ue ** 2) + np.sum(ve ** 2))))

    errors = {
        "step": "first timed step; oracle inputs = the GPU's pre-step state (advection) and its advected faces (projections)",
        "hybrid_p_vs_oracle_same_algorithm": rel(gpu["p_hybrid"], o["p"]),
        "hybrid_p_vs_oracle_fp64_network": rel(gpu["p_hybrid"], o64["p"]),
        "hybrid_p_vs_exact_solve": rel(gpu["p_hybrid"], ex),
        "oracle_hybrid_p_vs_exact_solve": rel(o["p"], ex),
        "pcg_p_vs_exact_solve": rel(gpu["p_pcg"], ex),
        "hybrid_uv_vs_exact_projection": rel_uv(gpu["p_hybrid"]),
        "pcg_uv_vs_exact_projection": rel_uv(gpu["p_pcg"]),
        "oracle_pcg_p_vs_exact_solve": rel(o_pcg["p"], ex),
        "hybrid_sweeps": k, "oracle_pcg_iters": int(o_pcg["iters"]), "pcg_iters": gpu["pcg_iters"],
        "bars": "same-algorithm relative L2 of p: 1e-3 (BF16 network), 1e-4 (FP32)",
    }
    cpu = {"value": 1.0 / (t_adv + t_proj), "unit": "timesteps/s", "cores": int(cores), "kind": "oracle",
           "sample": (f"one FP64 oracle time step at 512^2 (the first timed step): advection "
                      f"{t_adv:.2f} s + hybrid replica (BF16-emulated 4-scale 64-channel network, "
                      f"{k} Jacobi sweeps) {t_proj:.2f} s; the oracle PCG on the same faces took "
                      f"{t_pcg:.2f} s ({int(o_pcg['iters'])} iterations, "
                      f"{1.0 / (t_adv + t_pcg):.3f} timesteps/s); numpy stencils single-threaded, "
                      f"BLAS threads = cores")}
    return cpu, errors


def pct(a, q):
    return round(float(np.percentile(np.asarray(a, dtype=np.float64), q)), 4)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--check-every", type=int, default=CHECK_EVERY["hybrid"],
                    help="sweeps between the hybrid's E_1 tests")
    args = ap.parse_args()
    CHECK_EVERY["hybrid"] = args.check_every
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only; multi-GPU sharding is a design "
              "note, not a code path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import scenes
    import paper_2109_09363_amd as hp

    dev = torch.device("cuda")
    sc = scenes.plume_scene(N, seed=0, n_obstacles=(0, 3))
    w_np, w_kind = load_weights(scenes)
    K, W = args.steps, args.warmup
    noise = np.stack([scenes.inflow_noise(0, s, N) for s in range(W + K)]).astype(np.float32)
    xi = torch.from_numpy(noise).to(dev)
    flags = torch.from_numpy(sc.flags).to(dev)
    weights = torch.from_numpy(w_np).to(dev)

    pr = hp.Projector(N, N, sc.dx, 1.0, sc.rho0, SCALES, CHANNELS, "bf16")
    pr.set_weights(weights)
    pr.plan(flags)
    rho = torch.full((N, N), sc.rho0, dtype=torch.float32, device=dev)
    u = torch.zeros((N, N + 1), dtype=torch.float32, device=dev)
    v = torch.zeros((N + 1, N), dtype=torch.float32, device=dev)
    p = torch.zeros((N, N), dtype=torch.float32, device=dev)

    def step(method, s, x=None):
        pr.step_async(rho, u, v, flags, p, xi[s] if x is None else x, THRESHOLD, g=sc.g,
                      drho=sc.drho, u_in=sc.u_in, cfl=0.5, method=method, max_iters=MAX_ITERS,
                      check_every=CHECK_EVERY[method])

    print(f"# warmup {W} PCG steps", file=sys.stderr, flush=True)
    for s in range(W):
        step("pcg", s)
    torch.cuda.synchronize()
    snap = [t.clone() for t in (rho, u, v, p)]

    def restore():
        for dst, src in zip((rho, u, v, p), snap):
            dst.copy_(src)
        torch.cuda.synchronize()

    # each method's time step captured once as a hipGraph (the persistent
    # solver becomes a plain launch of the same grid) and replayed per step
    # with that step's inflow noise copied into the captured buffer
    xb = torch.empty_like(xi[0])
    graphs = {}
    for method in ("hybrid", "pcg"):
        restore()
        graphs[method] = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graphs[method]):
            step(method, None, x=xb)
        torch.cuda.synchronize()

    def timed(method):
        restore()
        t0 = time.perf_counter()
        for s in range(W, W + K):
            xb.copy_(xi[s])
            graphs[method].replay()
        torch.cuda.synchronize()
        return time.perf_counter() - t0

    print(f"# timing {K} hybrid steps", file=sys.stderr, flush=True)
    t_h = timed("hybrid")
    last_h = pr.result()
    print(f"# timing {K} pcg steps", file=sys.stderr, flush=True)
    t_p = timed("pcg")
    last_p = pr.result()

    # instrumented replays: per-step results and library phase timing
    def instrumented(method):
        restore()
        pr.set_timing(True)
        rows = []
        for s in range(W, W + K):
            step(method, s)
            torch.cuda.synchronize()
            r = pr.result()
            rows.append((r, pr.timing()))
        pr.set_timing(False)
        return rows

    print("# instrumented replays", file=sys.stderr, flush=True)
    rows_h = instrumented("hybrid")
    rows_p = instrumented("pcg")
    it_h = np.array([r.iters for r, _ in rows_h], dtype=np.float64)
    it_p = np.array([r.iters for r, _ in rows_p], dtype=np.float64)
    st_h = [r.status for r, _ in rows_h]
    solver_ms = np.array([t["solver"] for _, t in rows_h])
    inf_ms = np.array([t["inference"] for _, t in rows_h])
    adv_ms = np.array([t["advect"] for _, t in rows_h])
    tot_ms = np.array([t["total"] for _, t in rows_h])
    e1f = max(r.e1_final for r, _ in rows_h)

    # roofline of the dominant kernel: the persistent Jacobi launch (one per
    # projection; the solver phase's HIP events bracket exactly that launch)
    cells = N * N
    bytes_per_launch = float(BYTES_PER_CELL_SWEEP * cells * it_h.mean())
    avg_ms = float(solver_ms.mean())
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if avg_ms > 0 else 0.0
    traffic, traffic_src = measured_traffic()
    dram = None if traffic is None or avg_ms <= 0 else traffic / (avg_ms * 1e-3) / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None if traffic is None else round(traffic),
                "traffic_source": traffic_src,
                "kernel": "jacobi_reg", "avg_launch_ms": round(avg_ms, 4),
                "algorithmic_bytes_per_launch": round(bytes_per_launch),
                "bytes_per_cell_sweep": BYTES_PER_CELL_SWEEP,
                "regime": ("synchronisation latency: the 1 MB state stays in registers between tile "
                           "exchanges, so achieved counts algorithmic bytes (13 B/cell/sweep), not DRAM "
                           "traffic, and can exceed the HBM peak (frac > 1); dram_gbs is the counted "
                           "DRAM traffic; the DRAM-resident streaming kernel is measured at 8192^2 "
                           "separately"),
                "dram_gbs": None if dram is None else round(dram, 1),
                "dram_frac": None if dram is None else round(dram / HBM_PEAK_GBS, 4)}

    cpu, errors = None, None
    if not args.no_cpu:
        # the first timed step once more: its advected faces (the advection
        # is deterministic), then each method's step, for the oracle leg
        print("# first timed step for the oracle comparison", file=sys.stderr, flush=True)
        f64 = lambda t: t.cpu().numpy().astype(np.float64)
        restore()
        pre = (f64(rho), f64(u), f64(v), f64(xi[W]))
        pr.advect_async(rho, u, v, xi[W], g=sc.g, drho=sc.drho, u_in=sc.u_in, cfl=0.5)
        torch.cuda.synchronize()
        ustar = (f64(u), f64(v))
        gpu = {}
        for method in ("hybrid", "pcg"):
            restore()
            step(method, W)
            torch.cuda.synchronize()
            r = pr.result()
            gpu["p_" + method] = f64(p)
            gpu[method + "_iters"] = int(r.iters)
            gpu["dt"] = float(r.dt)
        print("# cpu oracle baseline and errors", file=sys.stderr, flush=True)
        cpu, errors = oracle_leg(sc, sc.flags, pre, ustar, gpu, w_np)

    value = K / t_h
    out = {
        "metric": "timesteps/s at 512², mean|div|<=1e-3: CNN+Jacobi vs PCG on same GPU; HBM GB/s",
        "value": round(value, 3), "unit": "timesteps/s", "n_gpus": 1, "steps": K, "warmup": W,
        "ms_per_step": round(1e3 * t_h / K, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": ("512x512 plume, 0-3 disks (seed 0), developed by PCG-projected steps; hybrid "
                                "4-scale 64-ch BF16 CNN + FP32 Jacobi to mean|div|<1e-3 (E_1 tested every %d "
                                "sweeps; PCG every iteration), per full time step incl. advection"
                                % CHECK_EVERY["hybrid"]),
                   "plume_age_steps": W,
                   "launch": "each method's time step captured once as a hipGraph and replayed per step",
                   "cnn_dtype": "bf16", "solver_dtype": "f32", "weights": w_kind,
                   "n_obstacles": len(sc.disks), "threshold": THRESHOLD},
        "hybrid": {"timesteps_per_s": round(value, 3), "mean_sweeps": round(float(it_h.mean()), 1),
                   "max_sweeps": int(it_h.max()), "statuses": sorted(set(st_h)),
                   "t_ad_ms": round(float(np.median(adv_ms)), 4), "t_inf_ms": round(float(np.median(inf_ms)), 4),
                   "t_solver_ms": round(float(np.median(solver_ms)), 4), "t_it_ms": round(float(np.median(tot_ms)), 4),
                   "projections_per_s": round(float(1e3 / np.mean(tot_ms - adv_ms)), 2),
                   "max_e1_final": e1f,
                   "timed_last_step": {"status": last_h.status, "iters": last_h.iters,
                                       "e1_final": last_h.e1_final},
                   "ms_per_step_p10_p50_p90": [pct(tot_ms, 10), pct(tot_ms, 50), pct(tot_ms, 90)],
                   "sweeps_p10_p50_p90": [pct(it_h, 10), pct(it_h, 50), pct(it_h, 90)]},
        "pcg": {"timesteps_per_s": round(K / t_p, 3), "mean_iters": round(float(it_p.mean()), 1),
                "max_iters": int(it_p.max()), "statuses": sorted(set(r.status for r, _ in rows_p)),
                "max_e1_final": max(r.e1_final for r, _ in rows_p),
                "timed_last_step": {"status": last_p.status, "iters": last_p.iters,
                                    "e1_final": last_p.e1_final},
                "t_solver_ms": round(float(np.median([t["solver"] for _, t in rows_p])), 4),
                "us_per_iteration": round(1e3 * float(np.sum([t["solver"] for _, t in rows_p])) /
                                          max(float(it_p.sum()), 1.0), 3),
                "ms_per_step_p10_p50_p90": [pct([t["total"] for _, t in rows_p], q) for q in (10, 50, 90)]},
        "hybrid_over_pcg": round(t_p / t_h, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "error_vs_fp64_oracle": errors,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
