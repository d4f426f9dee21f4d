"""Fixed workloads for rocprofv3 (kernel trace and PMC counter passes).

python -m paper_2109_09363_amd.profile_run WHAT [--n 512] [--sweeps 4096] [--reps 3]

WHAT:
  jacobi   fixed Jacobi sweeps on a 512^2 plume state (the hybrid's solver)
  pcg      fixed PCG iterations on the same state
  cnn      CNN inference only (4 scales, 64 channels, BF16)
  copy     a device-to-device copy of 256 MiB (calibration of FETCH/WRITE_SIZE)
  batch    one batched projection of many uneven plumes (streaming Jacobi)
  dram     the streaming Jacobi on one --n x --n grid (default 8192^2), fixed sweeps
Each workload runs once untimed, then `reps` times; the launch count and the
algorithmic bytes of one launch are printed so that per-dispatch counters can
be compared with them.
"""
from __future__ import annotations

import argparse
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


def plume_state(n, dev, steps=10):
    """A developed plume: `steps` PCG-projected time steps from rest; returns
    the projector, flags and an advected (not yet projected) u*, v*."""
    sc = scenes.plume_scene(n, seed=0, n_obstacles=(0, 3))
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0, 4, 64, "bf16", device=dev)
    w = np.load(WEIGHTS) if os.path.exists(WEIGHTS) else scenes.random_weights(4, 64, 0, 0.0)
    tw = torch.from_numpy(w.astype(np.float32)).to(dev)
    pr.set_weights(tw)
    flags = torch.from_numpy(sc.flags).to(dev)
    pr.plan(flags)
    rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device=dev)
    u = torch.zeros((n, n + 1), dtype=torch.float32, device=dev)
    v = torch.zeros((n + 1, n), dtype=torch.float32, device=dev)
    p = torch.zeros((n, n), dtype=torch.float32, device=dev)
    for s in range(steps):
        xi = torch.from_numpy(scenes.inflow_noise(0, s, n).astype(np.float32)).to(dev)
        pr.step_async(rho, u, v, flags, p, xi, 1e-3, g=sc.g, drho=sc.drho, method="pcg",
                      max_iters=20000)
    xi = torch.from_numpy(scenes.inflow_noise(0, steps, n).astype(np.float32)).to(dev)
    pr.advect_async(rho, u, v, xi, g=sc.g, drho=sc.drho)
    torch.cuda.synchronize()
    return pr, flags, u, v, p, tw


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["jacobi", "pcg", "cnn", "copy", "batch", "dram"])
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--sweeps", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--check-every", type=int, default=None,
                    help="batch, dram: E_1 test interval (default: only at the end)")
    a = ap.parse_args()
    if a.check_every is None:
        a.check_every = max(a.sweeps, 1)
    dev = torch.device("cuda")
    n = a.n
    if a.what == "copy":
        nbytes = 256 << 20
        src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).uniform_()
        dst = torch.empty_like(src)
        for _ in range(a.reps + 1):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"copy: {a.reps + 1} launches, {nbytes} B read + {nbytes} B written per launch")
        return
    if a.what == "batch":
        sides = [128, 192, 256, 384, 512]
        rng = np.random.default_rng(0)
        inst = []
        for i in range(32):
            s = int(rng.choice(sides))
            sc = scenes.plume_scene(s, seed=100 + i, n_obstacles=(0, 3))
            u, v = scenes.random_faces(s, s, 100 + i, kind="mixed")
            inst.append(dict(nx=s, ny=s, dx=sc.dx, flags=torch.from_numpy(sc.flags).to(dev),
                             u=torch.from_numpy(u.astype(np.float32)).to(dev),
                             v=torch.from_numpy(v.astype(np.float32)).to(dev),
                             p=torch.zeros((s, s), dtype=torch.float32, device=dev)))
        b = hp.Batch(inst, threshold=0.0, method="jacobi", max_iters=a.sweeps,
                     check_every=a.check_every)
        cells = sum(d["nx"] * d["ny"] for d in inst)
        for _ in range(a.reps + 1):
            b.project_async()
        torch.cuda.synchronize()
        print(f"batch: {len(inst)} instances, {cells} cells, {a.sweeps} sweeps per launch, "
              f"algorithmic bytes per launch {13 * cells * a.sweeps}")
        return
    if a.what == "dram":
        sc = scenes.plume_scene(n, seed=0, n_obstacles=2)
        u, v = scenes.random_faces(n, n, 0, kind="white")
        inst = [dict(nx=n, ny=n, dx=sc.dx, flags=torch.from_numpy(sc.flags).to(dev),
                     u=torch.from_numpy(u.astype(np.float32)).to(dev),
                     v=torch.from_numpy(v.astype(np.float32)).to(dev),
                     p=torch.zeros((n, n), dtype=torch.float32, device=dev))]
        b = hp.Batch(inst, threshold=0.0, method="jacobi", max_iters=a.sweeps,
                     check_every=a.check_every)
        for _ in range(a.reps + 1):
            b.project_async()
        torch.cuda.synchronize()
        print(f"dram: {a.reps + 1} projections of {a.sweeps} sweeps at {n}^2 (E_1 tested every "
              f"{a.check_every}); algorithmic bytes per jacobi_batch launch {13 * n * n * a.sweeps}")
        return
    pr, flags, u, v, p, tw = plume_state(n, dev)
    uu, vv = u.clone(), v.clone()
    if a.what == "cnn":
        for _ in range(a.reps + 1):
            uu.copy_(u); vv.copy_(v)
            pr.project_async(uu, vv, flags, p, 0.0, method="cnn")
        torch.cuda.synchronize()
        print(f"cnn: {a.reps + 1} inferences at {n}^2")
        return
    method = "jacobi" if a.what == "jacobi" else "pcg"
    t0 = time.perf_counter()
    for _ in range(a.reps + 1):
        uu.copy_(u); vv.copy_(v)
        pr.project_async(uu, vv, flags, p, 0.0, method=method, fixed_iters=a.sweeps)
    torch.cuda.synchronize()
    per = 13 if method == "jacobi" else 47
    print(f"{method}: {a.reps + 1} launches of {a.sweeps} iterations at {n}^2 "
          f"({time.perf_counter() - t0:.3f} s); algorithmic bytes per launch "
          f"{per * n * n * a.sweeps}")


if __name__ == "__main__":
    main()
