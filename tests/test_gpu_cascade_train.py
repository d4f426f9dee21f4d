"""Training of the paper's cascaded MultiScale and SmallScale networks
(Sec. 3.1, Fig. 3) with the solver in the loop (Sec. 3.2) on the GPU: the
hand-written adjoint (5x5 and 3x3 convolutions with the replicate-padding
adjoint, the up-sampled coarser output's transposed bilinear x2, the input
down-sampling adjoints) against the FP64 oracle gradient and against central
differences of the GPU's own loss, through the C ABI."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import cascade_adjoint as CA
from oracle import papernets as PN
from tests.gpu_util import to_dev, f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


class CascadeRun:
    def __init__(self, sc, arch):
        self.pr = hp.Projector(sc.nx, sc.ny, sc.dx, 1.0, 1.0, precision="fp32", arch=arch, train=True)
        self.tf = to_dev(sc.flags, torch.uint8)
        self.pr.plan(self.tf)

    def __call__(self, u, v, w, K, grads=True):
        pr = self.pr
        pr.set_weights(to_dev(w))
        tu, tv = to_dev(u), to_dev(v)
        p = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device="cuda")
        pr.project_async(tu, tv, self.tf, p, 0.0, method="hybrid" if K > 0 else "cnn", fixed_iters=K)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        du = torch.empty((pr.ny, pr.nx + 1), dtype=torch.float32, device="cuda") if grads else None
        dv = torch.empty((pr.ny + 1, pr.nx), dtype=torch.float32, device="cuda") if grads else None
        dp = torch.empty(pr.param_count, dtype=torch.float32, device="cuda") if grads else None
        pr.backward_async(K, 1.0, 1.0, du=du, dv=dv, dparams=dp, loss=loss)
        torch.cuda.synchronize()
        out = dict(loss=float(loss.item()))
        if grads:
            out.update(du=du.cpu().numpy().astype(np.float64), dv=dv.cpu().numpy().astype(np.float64),
                       dp=dp.cpu().numpy().astype(np.float64))
        return out


def case(arch, n, seed, nobs):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    w = f32(scenes.random_paper_weights(arch, seed))
    return sc, f32(u), f32(v), w


@pytest.mark.parametrize("arch,n,K,seed,nobs", [("smallscale", 32, 0, 0, 1), ("smallscale", 64, 6, 1, 2),
                                                ("multiscale", 64, 4, 2, 2), ("multiscale", 128, 3, 3, 3)])
def test_cascade_backward_matches_oracle(arch, n, K, seed, nobs):
    """Random weights: a few units within FP32 rounding of a ReLU kink take
    the other branch on the GPU, so the bar is 1e-3 (relative L2)."""
    say("cascade adjoint", arch, n, K)
    sc, u, v, w = case(arch, n, seed, nobs)
    g = CascadeRun(sc, arch)(u, v, w, K)
    loss, gu, gv, gp = CA.loss_and_grad(sc.flags, u, v, sc.dx, w.astype(np.float64), arch, K)
    ep, eu, ev = rel_l2(g["dp"], gp), rel_l2(g["du"], gu), rel_l2(g["dv"], gv)
    say(f"  loss {g['loss']:.8e} vs {loss:.8e}; rel L2 dparams {ep:.2e} du {eu:.2e} dv {ev:.2e}")
    assert g["loss"] == pytest.approx(loss, rel=1e-5)
    assert ep <= 1e-3 and eu <= 1e-3 and ev <= 1e-3
    # every branch's parameters, not only the total
    o = 0
    for b, br in enumerate(PN.branches(arch)):
        m = sum(k * k * ci * co + co for (k, ci, co, _r) in br)
        eb = rel_l2(g["dp"][o:o + m], gp[o:o + m])
        say(f"  branch {b}: rel L2 {eb:.2e}")
        assert eb <= 2e-3
        o += m


def test_cascade_gradient_matches_its_own_central_differences():
    """The GPU's gradient of the finest branch's 1x1 head (where the loss is a
    smooth quadratic) against central differences of the GPU's FP64-reduced
    loss, per weight and for the bias."""
    arch = "smallscale"
    sc, u, v, w = case(arch, 32, 3, 1)
    run = CascadeRun(sc, arch)
    g = run(u, v, w, 3)
    for i in list(range(w.size - 33, w.size - 29)) + [w.size - 1]:
        h = 2.0 ** -5
        wp, wm = f32(w.copy()), f32(w.copy())
        wp[i] = f32(w[i] + h)
        wm[i] = f32(w[i] - h)
        h = 0.5 * (wp[i] - wm[i])
        fd = (run(u, v, wp, 3, grads=False)["loss"] - run(u, v, wm, 3, grads=False)["loss"]) / (2 * h)
        say("  param", i, "fd", fd, "adjoint", g["dp"][i])
        assert g["dp"][i] == pytest.approx(fd, rel=1e-4, abs=1e-7 * abs(g["loss"]))


def test_cascade_training_gain():
    """Solver-in-the-loop training of SmallScale on plume states and
    divergence sources (train.py, FP32, 64^2): the loss falls, and on
    held-out plume states the trained network's guess leaves the hybrid
    fewer sweeps than no guess (plain Jacobi)."""
    from paper_2109_09363_amd import train as TR
    n, arch = 64, "smallscale"
    data = TR.generate_dataset(n, n_scenes=6, steps=20, keep_every=2, n_random=24, seed=5, log=say)
    w, hist = TR.train(data, n, 0, 0, "fp32", steps=300, batch=4, lr=1e-3, sweeps=8, seed=2,
                       log=say, log_every=50, arch=arch)
    say("loss history", hist)
    # single-batch losses are noisy: the mean of the last three logged ones
    assert np.mean([h[1] for h in hist[-3:]]) < 0.5 * hist[0][1]
    held = TR.plume_states(n, 6, 30, seed=777)
    zero = w.copy()
    zero[-33:] = 0.0  # the finest branch's output layer 0: the guess is 0, plain Jacobi
    it_t, mx_t = TR.evaluate(held, n, 0, 0, "fp32", w, arch=arch)
    it_z, mx_z = TR.evaluate(held, n, 0, 0, "fp32", zero, arch=arch)
    say("held-out mean sweeps to 1e-3: trained SmallScale", it_t, "zero output", it_z)
    assert it_t < it_z
