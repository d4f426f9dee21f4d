"""Solver-in-the-loop training of the multi-scale CNN (or of the paper's own
networks, --arch multiscale / smallscale / unet, FP32) on the GPU.

The physics-driven loss of Sec. 3.2: the divergence left in the corrected
velocity, here after the CNN guess and K Jacobi sweeps (the hybrid's own
iteration), with the gradient of the correction (Eq. 2) and of the sweeps
taken by the library's adjoint.  Each sample's loss is normalised by its
initial divergence energy, so  loss = sum_F r^2 / sum_F d^2.  With --beta the
long-term term is added: the same loss after 4 (or, one time in ten, 16)
unrolled time steps of the plume with the network in the loop, the advection
not differentiated (Sec. 3.2, Fig. 5, Eq. 4).

Training data (the paper's Mantaflow set is not available): intermediate
velocities u* of plume runs that the plain solver (PCG) projects, on random
obstacle layouts with Ri in {0, 0.1}, plus random smooth and noisy
divergence fields on random obstacle layouts (the "divergence sources" of
the paper's training set).  Everything runs through the C ABI: advection,
projection, CNN forward/backward and Adam.

python -m paper_2109_09363_amd.train --n 128 --scales 4 --channels 64 \
    --precision bf16 --steps 400 --out weights.npy
The paper's Unet (Sec. 3.1, Fig. 4), or its cascaded MultiScale (Fig. 3):
python -m paper_2109_09363_amd.train --arch unet --n 128 --precision fp32 \
    --steps 600 --sweeps 16 --eval 8 --out unet.npy
Fine-tuning at the benchmark resolution from existing weights, judged by the
Jacobi sweeps the hybrid needs to reach a threshold on held-out plume states:
python -m paper_2109_09363_amd.train --n 512 --init w.npy --random 0 \
    --sweeps 64 --eval 6 --out w512.npy
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

import scenes
from . import api


def _dev(a, dtype=torch.float32, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).to(device)


class Sample:
    """One training state on the device: the intermediate velocity u*, v*,
    the density and the plume's physics (for the unrolled steps of the
    long-term loss)."""
    __slots__ = ("flags", "u", "v", "rho", "g", "drho", "u_in", "seed")

    def __init__(self, flags, u, v, rho, g, drho, u_in, seed):
        self.flags, self.u, self.v, self.rho = flags, u, v, rho
        self.g, self.drho, self.u_in, self.seed = g, drho, u_in, seed


def generate_dataset(n: int, n_scenes: int = 12, steps: int = 32, keep_every: int = 2,
                     n_random: int = 64, seed: int = 0, device="cuda", log=print):
    """List of Samples on the device."""
    samples = []
    t0 = time.time()
    for i in range(n_scenes):
        sid = seed * 1000 + i
        sc = scenes.plume_scene(n, seed=sid, n_obstacles=(0, 3), ri=0.1 if i % 2 == 0 else 0.0)
        pr = api.Projector(n, n, sc.dx, 1.0, sc.rho0, device=device)
        tf = _dev(sc.flags, torch.uint8, device)
        pr.plan(tf)
        rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device=device)
        u = torch.zeros((n, n + 1), dtype=torch.float32, device=device)
        v = torch.zeros((n + 1, n), dtype=torch.float32, device=device)
        p = torch.zeros((n, n), dtype=torch.float32, device=device)
        g = sc.g if sc.ri > 0 else 0.0
        for s in range(steps):
            xi = _dev(scenes.inflow_noise(sid, s, n), device=device)
            pr.advect_async(rho, u, v, xi, g=g, drho=sc.drho, u_in=sc.u_in)
            if s >= 1 and s % keep_every == 0:
                samples.append(Sample(tf, u.clone(), v.clone(), rho.clone(), g, sc.drho, sc.u_in,
                                      sid * 100 + s))
            pr.project_async(u, v, tf, p, 1e-3, method="pcg", max_iters=20000)
    rng = np.random.default_rng(seed + 7)
    for i in range(n_random):
        sid = seed * 1000 + 500 + i
        sc = scenes.plume_scene(n, seed=sid, n_obstacles=(0, 3))
        kind = ("smooth", "mixed", "white")[i % 3]
        uu, vv = scenes.random_faces(n, n, int(rng.integers(1 << 30)), kind=kind)
        rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device=device)
        # the divergence sources have no density variation (Ri = 0)
        samples.append(Sample(_dev(sc.flags, torch.uint8, device), _dev(uu, device=device),
                              _dev(vv, device=device), rho, 0.0, sc.drho, sc.u_in, sid * 100))
    torch.cuda.synchronize()
    log(f"dataset: {len(samples)} samples at {n}x{n} in {time.time() - t0:.1f} s")
    return samples


def draw_unroll(rng, long_frac: float = 0.1, short: int = 4, long: int = 16) -> int:
    """Number of unrolled steps of the long-term loss: 16 one time in ten,
    else 4 (Sec. 3.2)."""
    return long if rng.random() < long_frac else short


def unrolled_backward(pr, smp: Sample, sweeps: int, n_unroll: int, alpha: float, beta: float,
                      norm_short: float, grads, xis, weight: float = 1.0, accumulate: bool = False,
                      loss_short=None, loss_long=None, p=None):
    """Enqueue the gradient of  alpha * short + beta * long  for one sample
    (Sec. 3.2, Fig. 5, Eq. 4) into `grads` (added when `accumulate`).

    short: sum_F r^2 / sum_F d^2 after the network's projection (CNN guess and
    `sweeps` Jacobi sweeps) of u*_t;  long: the same after n_unroll more time
    steps (advection and forces, then the same projection with the network
    frozen), with the advection not differentiated: only the last projection
    is back-propagated.  xis[j] is the inflow perturbation (device, nx) of
    unrolled step j.  Returns the long-term normalisation (host sync)."""
    method = "hybrid" if sweeps > 0 else "cnn"
    n = pr.nx
    if p is None:
        p = torch.empty((pr.ny, n), dtype=torch.float32, device=smp.u.device)
    pr.plan(smp.flags)
    uu, vv = smp.u.clone(), smp.v.clone()
    pr.project_async(uu, vv, smp.flags, p, 0.0, method=method, fixed_iters=sweeps)
    if alpha != 0.0:
        pr.backward_async(sweeps, 1.0, weight * alpha * norm_short, dparams=grads, loss=loss_short,
                          accumulate=accumulate)
        accumulate = True
    if beta == 0.0 or n_unroll == 0:
        return 0.0
    rr = smp.rho.clone()
    for j in range(n_unroll):
        pr.advect_async(rr, uu, vv, xis[j], g=smp.g, drho=smp.drho, u_in=smp.u_in)
        pr.project_async(uu, vv, smp.flags, p, 0.0, method=method, fixed_iters=sweeps)
    r = pr.result()
    norm_long = 1.0 / max(r.s * r.s * r.n_fluid, 1e-30)
    pr.backward_async(sweeps, 1.0, weight * beta * norm_long, dparams=grads, loss=loss_long,
                      accumulate=accumulate)
    return norm_long


def initial_weights(arch: str, scales: int, channels: int, seed: int):
    """Seeded random init with a small output layer (the first guesses stay
    near zero)."""
    if arch in ("unet", "multiscale", "smallscale"):
        return scenes.random_paper_weights(arch, seed, out_scale=0.1)
    return scenes.random_weights(scales, channels, seed, out_scale=0.1)


def train(samples, n: int, scales: int, channels: int, precision: str = "fp32",
          steps: int = 200, batch: int = 4, lr: float = 1e-3, sweeps: int = 4,
          params0=None, seed: int = 0, device="cuda", log=print, log_every: int = 20,
          alpha: float = 1.0, beta: float = 0.0, arch: str = "parallel", lr_end=None):
    """Adam on  alpha * short-term + beta * long-term  normalised divergence
    losses (beta = 0: the single-step loss); returns (params, loss history).
    lr_end: None keeps lr constant; otherwise the rate follows a cosine from
    lr at the first step to lr_end at the last (so that the returned weights
    are not those of a single noisy late step)."""
    dx = 1.0 / n
    pr = api.Projector(n, n, dx, 1.0, 1.0, scales, channels, precision, device=device, train=True,
                       arch=arch)
    if params0 is None:
        params0 = initial_weights(arch, scales, channels, seed)
    params = _dev(params0, device=device)
    m = torch.zeros_like(params)
    v2 = torch.zeros_like(params)
    grads = torch.zeros_like(params)
    pr.set_weights(params)
    # per-sample normalisation from the library's CNN input scale s: sum d^2 = s^2 nF
    norms = []
    pz = torch.empty((n, n), dtype=torch.float32, device=device)
    for smp in samples:
        pr.plan(smp.flags)
        uu, vv = smp.u.clone(), smp.v.clone()
        pr.project_async(uu, vv, smp.flags, pz, 0.0, method="cnn")
        r = pr.result()
        norms.append(1.0 / max(r.s * r.s * r.n_fluid, 1e-30))
    rng = np.random.default_rng(seed)
    ls_dev = torch.zeros(1, dtype=torch.float64, device=device)
    ll_dev = torch.zeros(1, dtype=torch.float64, device=device)
    hist = []
    t0 = time.time()
    for it in range(1, steps + 1):
        idx = rng.choice(len(samples), batch, replace=False)
        logging = it % log_every == 0 or it == 1 or it == steps
        acc_loss = 0.0
        for b, i in enumerate(idx):
            smp = samples[i]
            xis = []
            n_unroll = 0
            if beta != 0.0:
                n_unroll = draw_unroll(rng)
                xis = [_dev(scenes.inflow_noise(smp.seed, 1 + 1000 * it + j, n), device=device)
                       for j in range(n_unroll)]
            unrolled_backward(pr, smp, sweeps, n_unroll, alpha, beta, norms[i], grads, xis,
                              weight=1.0 / batch, accumulate=b > 0, loss_short=ls_dev,
                              loss_long=ll_dev, p=pz)
            if logging:
                acc_loss += (float(ls_dev.item()) if alpha != 0.0 else 0.0) + \
                            (float(ll_dev.item()) if beta != 0.0 else 0.0)
        lr_it = lr
        if lr_end is not None and steps > 1:
            lr_it = lr_end + 0.5 * (lr - lr_end) * (1.0 + math.cos(math.pi * (it - 1) / (steps - 1)))
        api.adam_async(params, grads, m, v2, it, lr=lr_it)
        if logging:
            hist.append((it, acc_loss))
            log(f"step {it:5d}  loss {acc_loss:.5f}  ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return params.cpu().numpy(), hist


def plume_states(n: int, n_scenes: int, steps: int, seed: int, device="cuda"):
    """Held-out evaluation states: u* of plume runs after `steps` PCG-projected
    steps (the state the hybrid would project next)."""
    out = []
    for i in range(n_scenes):
        sc = scenes.plume_scene(n, seed=seed + i, n_obstacles=(0, 3))
        pr = api.Projector(n, n, sc.dx, 1.0, sc.rho0, device=device)
        tf = _dev(sc.flags, torch.uint8, device)
        pr.plan(tf)
        rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device=device)
        u = torch.zeros((n, n + 1), dtype=torch.float32, device=device)
        v = torch.zeros((n + 1, n), dtype=torch.float32, device=device)
        p = torch.zeros((n, n), dtype=torch.float32, device=device)
        for s in range(steps + 1):
            xi = _dev(scenes.inflow_noise(seed + i, s, n), device=device)
            pr.advect_async(rho, u, v, xi, g=sc.g, drho=sc.drho, u_in=sc.u_in)
            if s == steps:
                out.append([tf, u.clone(), v.clone()])
                break
            pr.project_async(u, v, tf, p, 1e-3, method="pcg", max_iters=20000)
    torch.cuda.synchronize()
    return out


def evaluate(states, n: int, scales: int, channels: int, precision: str, params, thr: float = 1e-3,
             device="cuda", arch: str = "parallel"):
    """Mean and max Jacobi sweeps the hybrid needs to reach mean|div| < thr."""
    pr = api.Projector(n, n, 1.0 / n, 1.0, 1.0, scales, channels, precision, device=device, arch=arch)
    pr.set_weights(_dev(params, device=device))
    p = torch.empty((n, n), dtype=torch.float32, device=device)
    its = []
    for (tf, u, v) in states:
        pr.plan(tf)
        uu, vv = u.clone(), v.clone()
        pr.project_async(uu, vv, tf, p, thr, method="hybrid", max_iters=1000000, check_every=8)
        its.append(pr.result().iters)
    return float(np.mean(its)), int(np.max(its))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--scales", type=int, default=4)
    ap.add_argument("--channels", type=int, default=64)
    ap.add_argument("--precision", default="bf16")
    ap.add_argument("--steps", type=int, default=400)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-end", type=float, default=None,
                    help="cosine decay of the rate to this value at the last step (default: constant)")
    ap.add_argument("--sweeps", type=int, default=4)
    ap.add_argument("--scenes", type=int, default=12)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--init", default=None, help="start from these weights (.npy)")
    ap.add_argument("--random", type=int, default=64, help="random divergence samples")
    ap.add_argument("--sim-steps", type=int, default=32, help="plume steps per scene")
    ap.add_argument("--eval", type=int, default=0, help="held-out plume states to evaluate")
    ap.add_argument("--eval-steps", type=int, default=40)
    ap.add_argument("--alpha", type=float, default=1.0, help="weight of the short-term loss")
    ap.add_argument("--beta", type=float, default=0.0,
                    help="weight of the long-term loss (4 or 16 unrolled steps)")
    ap.add_argument("--arch", default="parallel", choices=["parallel", "multiscale", "smallscale", "unet"])
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    params0 = None
    if a.init:
        params0 = np.load(a.init, allow_pickle=False).astype(np.float32)
    held = plume_states(a.n, a.eval, a.eval_steps, seed=900000 + a.seed) if a.eval > 0 else []
    if held and params0 is not None:
        m, mx = evaluate(held, a.n, a.scales, a.channels, a.precision, params0, arch=a.arch)
        print(f"eval before: mean sweeps to 1e-3 {m:.1f} (max {mx}) on {len(held)} held-out states",
              flush=True)
    data = generate_dataset(a.n, n_scenes=a.scenes, steps=a.sim_steps, n_random=a.random, seed=a.seed)
    w, hist = train(data, a.n, a.scales, a.channels, a.precision, steps=a.steps, batch=a.batch,
                    lr=a.lr, sweeps=a.sweeps, seed=a.seed, params0=params0, alpha=a.alpha,
                    beta=a.beta, arch=a.arch, lr_end=a.lr_end)
    if held:
        m, mx = evaluate(held, a.n, a.scales, a.channels, a.precision, w, arch=a.arch)
        print(f"eval after: mean sweeps to 1e-3 {m:.1f} (max {mx}) on {len(held)} held-out states",
              flush=True)
    if a.out:
        np.save(a.out, w.astype(np.float32), allow_pickle=False)
        print(f"saved {a.out}")


if __name__ == "__main__":
    main()
