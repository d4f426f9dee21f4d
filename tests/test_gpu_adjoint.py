"""GPU adjoint of the hybrid projection against the FP64 oracle gradient and
against finite differences of the GPU's own loss."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import adjoint as AJ
from oracle import cnn as CN
from tests.gpu_util import to_dev, f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


class Run:
    """Forward + backward on the GPU through the C ABI."""

    def __init__(self, sc, S, C, prec="fp32"):
        self.sc = sc
        self.pr = hp.Projector(sc.nx, sc.ny, sc.dx, 1.0, 1.0, S, C, prec, train=True)
        self.tf = to_dev(sc.flags, torch.uint8)
        self.pr.plan(self.tf)
        self.S, self.C = S, C

    def __call__(self, u, v, w, K, omega=1.0, scale=1.0, grads=True):
        pr = self.pr
        tw = to_dev(w)
        pr.set_weights(tw)
        tu, tv = to_dev(u), to_dev(v)
        p = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device="cuda")
        pr.project_async(tu, tv, self.tf, p, 0.0, method="hybrid" if K > 0 else "cnn",
                         fixed_iters=K, omega=omega)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        du = torch.empty((pr.ny, pr.nx + 1), dtype=torch.float32, device="cuda") if grads else None
        dv = torch.empty((pr.ny + 1, pr.nx), dtype=torch.float32, device="cuda") if grads else None
        dp = torch.empty(pr.param_count, dtype=torch.float32, device="cuda") if grads else None
        pr.backward_async(K, omega, scale, du=du, dv=dv, dparams=dp, loss=loss)
        torch.cuda.synchronize()
        out = dict(loss=float(loss.item()))
        if grads:
            out.update(du=du.cpu().numpy().astype(np.float64), dv=dv.cpu().numpy().astype(np.float64),
                       dp=dp.cpu().numpy().astype(np.float64))
        return out


def state(n, seed, nobs, ny=None):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs, ny=ny)
    u, v = scenes.random_faces(sc.nx, sc.ny, seed, kind="mixed")
    return sc, f32(u), f32(v)


@pytest.mark.parametrize("n,ny,S,C,K,omega,seed", [
    (32, None, 2, 16, 0, 1.0, 0), (32, None, 2, 16, 5, 1.0, 1), (48, 32, 3, 16, 7, 0.8, 2),
    (64, None, 3, 32, 20, 1.0, 3)])
def test_backward_matches_oracle(n, ny, S, C, K, omega, seed):
    say("adjoint", n, ny, S, C, K)
    sc, u, v = state(n, seed, 2, ny)
    w = f32(scenes.random_weights(S, C, seed))
    g = Run(sc, S, C)(u, v, w, K, omega)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K, omega)
    say("  loss", g["loss"], loss)
    say("  rel L2 dparams", rel_l2(g["dp"], gp), "du", rel_l2(g["du"], gu), "dv", rel_l2(g["dv"], gv))
    assert g["loss"] == pytest.approx(loss, rel=1e-5)
    assert rel_l2(g["dp"], gp) <= 1e-4
    assert rel_l2(g["du"], gu) <= 1e-4
    assert rel_l2(g["dv"], gv) <= 1e-4


@pytest.mark.parametrize("n,S,C,K,seed", [(64, 3, 32, 4, 4), (128, 4, 64, 8, 6)])
def test_backward_bf16_matches_emulated_oracle(n, S, C, K, seed):
    """The BF16 network's gradient (what training with --precision bf16
    uses) against the oracle's gradient of the same BF16-emulated forward
    with the straight-through reverse pass (rounded activations, unrounded
    weights): differences come from FP32 against FP64 accumulation and the
    few roundings that the two take differently; the unemulated FP64
    gradient is further away."""
    sc, u, v = state(n, seed, 2)
    w = f32(scenes.random_weights(S, C, seed))
    g = Run(sc, S, C, "bf16")(u, v, w, K)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K, bf16=True)
    _l64, gu64, _gv64, gp64 = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K)
    ep, eu, ev = rel_l2(g["dp"], gp), rel_l2(g["du"], gu), rel_l2(g["dv"], gv)
    say(f"  bf16 vs emulated: dparams {ep:.2e} du {eu:.2e} dv {ev:.2e}; vs FP64 network: dparams "
        f"{rel_l2(g['dp'], gp64):.2e} du {rel_l2(g['du'], gu64):.2e}; loss {g['loss']:.6e} vs {loss:.6e}")
    assert g["loss"] == pytest.approx(loss, rel=1e-3)
    assert ep <= 1e-2 and eu <= 1e-2 and ev <= 1e-2


def test_backward_deterministic_and_accumulate():
    sc, u, v = state(64, 5, 2)
    w = f32(scenes.random_weights(3, 16, 5))
    r = Run(sc, 3, 16)
    a = r(u, v, w, 6)
    b = r(u, v, w, 6)
    assert np.array_equal(a["dp"], b["dp"]) and np.array_equal(a["du"], b["du"])
    # accumulate adds onto the existing gradient
    pr = r.pr
    dp = torch.from_numpy(a["dp"].astype(np.float32)).cuda()
    pr.backward_async(6, 1.0, 1.0, dparams=dp, accumulate=True)
    torch.cuda.synchronize()
    assert np.allclose(dp.cpu().numpy(), 2 * a["dp"], rtol=1e-6, atol=0)


def snap(x, bits=20):
    return np.round(np.asarray(x, np.float64) * 2.0 ** bits) / 2.0 ** bits


def test_fd_head_parameters_exact_quadratic():
    # the loss is exactly quadratic in the 1x1 head (no ReLU after it): the
    # central difference has no truncation error, only FP32 rounding
    S, C, K = 3, 16, 10
    sc, u, v = state(64, 6, 1)
    w = snap(scenes.random_weights(S, C, 6))
    run = Run(sc, S, C)
    g = run(u, v, w, K)
    rng = np.random.default_rng(0)
    dirn = np.zeros_like(w)
    per = CN.param_count(1, C)
    for k in range(S):
        o = k * per + per - (C + 1)
        dirn[o:o + C + 1] = rng.choice([-1.0, 1.0], C + 1)
    gd = float(g["dp"] @ dirn)
    for h, tol in ((2.0 ** -10, 1e-3), (2.0 ** -3, 1e-5)):
        lp = run(u, v, w + h * dirn, K, grads=False)["loss"]
        lm = run(u, v, w - h * dirn, K, grads=False)["loss"]
        fd = (lp - lm) / (2 * h)
        say("  head FD h", h, fd, "adjoint", gd)
        assert fd == pytest.approx(gd, rel=tol)


def test_fd_velocity_with_zero_network_exact_quadratic():
    # zero weights: phi0 = 0 and the loss is a quadratic form of u, v
    S, C, K = 3, 16, 12
    sc, u, v = state(64, 7, 2)
    u, v = snap(u), snap(v)
    w = np.zeros(CN.param_count(S, C))
    run = Run(sc, S, C)
    g = run(u, v, w, K)
    rng = np.random.default_rng(1)
    du = rng.choice([-1.0, 1.0], u.shape)
    dv = rng.choice([-1.0, 1.0], v.shape)
    gd = float(np.sum(g["du"] * du) + np.sum(g["dv"] * dv))
    for h, tol in ((2.0 ** -10, 1e-3), (2.0 ** -4, 1e-5)):
        lp = run(u + h * du, v + h * dv, w, K, grads=False)["loss"]
        lm = run(u - h * du, v - h * dv, w, K, grads=False)["loss"]
        fd = (lp - lm) / (2 * h)
        say("  velocity FD h", h, fd, "adjoint", gd)
        assert fd == pytest.approx(gd, rel=tol)


def test_autograd_function():
    S, C, K = 2, 16, 3
    sc, u, v = state(32, 8, 1)
    w = f32(scenes.random_weights(S, C, 8))
    pr = hp.Projector(32, 32, sc.dx, 1.0, 1.0, S, C, "fp32", train=True)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    tu = to_dev(u).requires_grad_(True)
    tv = to_dev(v).requires_grad_(True)
    tw = to_dev(w).requires_grad_(True)
    loss = hp.ProjectionLoss.apply(tu, tv, tw, pr, tf, K, 1.0, 0.5)
    (3.0 * loss).backward()
    l0, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K, 1.0, 0.5)
    assert float(loss) == pytest.approx(l0, rel=1e-5)
    assert rel_l2(tw.grad.cpu().numpy(), 3 * gp) <= 1e-4
    assert rel_l2(tu.grad.cpu().numpy(), 3 * gu) <= 1e-4


def test_checkpoints_replay_bitwise():
    # phi after every 5 of the K = 20 forward sweeps.  The sweep is affine in
    # phi, so the adjoint needs none of these iterates; restarting from a
    # checkpoint as a warm start reproduces the later ones bit for bit.
    from oracle import grid as G
    from oracle import solve as SV
    n, K, c = 256, 20, 5
    sc, u, v = state(n, 9, 2)
    pr = hp.Projector(n, n, sc.dx, 1.0, 1.0, 0, 0, "fp32")
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    ck = torch.empty((K // c, n, n), dtype=torch.float32, device="cuda")
    p = torch.empty((n, n), dtype=torch.float32, device="cuda")
    pr.project_async(to_dev(u), to_dev(v), tf, p, 0.0, method="jacobi", fixed_iters=K,
                     checkpoint_every=c, phi_ckpt=ck)
    torch.cuda.synchronize()
    assert torch.equal(ck[-1], p)  # dt = rho0 = 1 and no folds: p is the last iterate
    for i in range(K // c - 1):
        p2 = torch.empty_like(p)
        pr.project_async(to_dev(u), to_dev(v), tf, p2, 0.0, method="jacobi", fixed_iters=c,
                         p_init=ck[i].clone())
        torch.cuda.synchronize()
        assert torch.equal(p2, ck[i + 1]), i
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    phi5 = SV.jacobi(P, d, sc.dx, np.zeros(P.shape), fixed_iters=c)[0]
    err = rel_l2(ck[0].cpu().numpy().astype(np.float64), phi5, P.fluid)
    say("  checkpoint 0 vs oracle 5 sweeps", err)
    assert err <= 1e-5
