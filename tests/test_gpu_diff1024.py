"""The differentiation workload at full size: a 1024x1024 plume with two
obstacles, the 3-scale 32-channel FP32 network, loss = sum of squared
divergence after the CNN guess and 20 Jacobi sweeps.  The GPU adjoint's
gradients w.r.t. the input velocity and the weights are compared with the
FP64 oracle gradient, on the whole field and on two 32x32 windows (an
obstacle edge and the inflow), and with central finite differences of the
GPU loss.

At a million pixels some hidden pre-activations sit within FP32 rounding of
a ReLU kink, where FP32 and FP64 can take different branches (tests/kinks.py).
So the whole-field comparison runs twice: with weights whose biases keep every
unit strictly active (no decision is close; every face compared), and with
plain random weights, where the faces reachable from a unit within 2e-6 A of
its kink are left out (a single FP32 convolution was measured at most 5e-7 A
from FP64 on these inputs)."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import adjoint as AJ
from oracle import cnn as CN
from oracle import grid as G
from tests import kinks
from tests.gpu_util import to_dev, f32, rel_l2

pytestmark = pytest.mark.gpu

N, S, C, K = 1024, 3, 32, 20
TAU = 2e-6


def say(*a):
    print(*a, flush=True)


def window_at_obstacle_edge(P, size=32):
    solid = ~P.fluid
    edge = solid & (np.roll(P.fluid, 1, 0) | np.roll(P.fluid, -1, 0))
    jj, ii = np.nonzero(edge)
    j, i = int(jj[len(jj) // 2]), int(ii[len(ii) // 2])
    j0 = min(max(j - size // 2, 0), P.shape[0] - size)
    i0 = min(max(i - size // 2, 0), P.shape[1] - size)
    return slice(j0, j0 + size), slice(i0, i0 + size)


@pytest.fixture(scope="module")
def case():
    sc = scenes.plume_scene(N, seed=21, n_obstacles=2)
    u, v = scenes.random_faces(N, N, 21, kind="mixed")
    u, v = f32(u), f32(v)
    w = f32(scenes.random_weights(S, C, 21))
    P = G.plan(sc.flags)
    pr = hp.Projector(N, N, sc.dx, 1.0, 1.0, S, C, "fp32", train=True)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)

    def run(uu, vv, ww, grads=True):
        pr.set_weights(to_dev(ww))
        tu, tv = to_dev(uu), to_dev(vv)
        p = torch.empty((N, N), dtype=torch.float32, device="cuda")
        pr.project_async(tu, tv, tf, p, 0.0, method="hybrid", fixed_iters=K)
        loss = torch.zeros(1, dtype=torch.float64, device="cuda")
        du = torch.empty((N, N + 1), dtype=torch.float32, device="cuda") if grads else None
        dv = torch.empty((N + 1, N), dtype=torch.float32, device="cuda") if grads else None
        dp = torch.empty(pr.param_count, dtype=torch.float32, device="cuda") if grads else None
        pr.backward_async(K, 1.0, 1.0, du=du, dv=dv, dparams=dp, loss=loss)
        torch.cuda.synchronize()
        out = dict(loss=float(loss.item()))
        if grads:
            out.update(du=du.cpu().numpy().astype(np.float64), dv=dv.cpu().numpy().astype(np.float64),
                       dp=dp.cpu().numpy().astype(np.float64))
        return out

    return sc, P, u, v, w, run


def test_gradients_match_fp64_oracle_all_units_active(case):
    sc, P, u, v, w, run = case
    wl = kinks.linear_regime(P, u, v, sc.dx, w, S, C)
    ratios = kinks.pre_activation_ratios(P, u, v, sc.dx, wl, S, C)
    say("linear regime: smallest |z|/A", min(r.min() for r in ratios))
    assert min(r.min() for r in ratios) >= 1e-3
    say("gpu forward + adjoint at 1024^2")
    g = run(u, v, wl)
    say("oracle FP64 gradient at 1024^2")
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, wl, S, C, K)
    say("loss", g["loss"], loss)
    assert g["loss"] == pytest.approx(loss, rel=1e-5)
    e_p, e_u, e_v = rel_l2(g["dp"], gp), rel_l2(g["du"], gu), rel_l2(g["dv"], gv)
    say("rel L2 dparams", e_p, "du", e_u, "dv", e_v)
    assert e_p <= 1e-4 and e_u <= 1e-4 and e_v <= 1e-4
    wj, wi = window_at_obstacle_edge(P)
    e_w = rel_l2(g["du"][wj, wi], gu[wj, wi])
    inflow = np.nonzero(P.vinflow)[0]
    ci = int(inflow[len(inflow) // 2])
    e_in = rel_l2(g["dv"][0:32, ci - 16:ci + 16], gv[0:32, ci - 16:ci + 16])
    say("32x32 windows: obstacle edge du", e_w, "inflow dv", e_in)
    assert e_w <= 1e-4 and e_in <= 1e-4


def test_gradients_match_fp64_oracle_away_from_kinks(case):
    sc, P, u, v, w, run = case
    g = run(u, v, w)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K)
    flagged = kinks.ambiguous_units(P, u, v, sc.dx, w, S, C, TAU)
    um, vm = kinks.kink_free_faces(flagged, N, N)
    say("units within", TAU, "A of a kink (pixels per scale):", [int(f.sum()) for f in flagged],
        "faces compared:", float(um.mean()), float(vm.mean()))
    e_p = rel_l2(g["dp"], gp)
    e_u, e_v = rel_l2(g["du"], gu, um), rel_l2(g["dv"], gv, vm)
    say("rel L2 dparams", e_p, "du (kink-free)", e_u, "dv (kink-free)", e_v,
        "whole field du", rel_l2(g["du"], gu), "dv", rel_l2(g["dv"], gv))
    assert g["loss"] == pytest.approx(loss, rel=1e-5)
    assert e_p <= 1e-4 and e_u <= 1e-4 and e_v <= 1e-4
    assert um.mean() >= 0.3 and vm.mean() >= 0.3


def test_fd_head_at_full_size(case):
    # the loss is exactly quadratic in the 1x1 heads (no ReLU after them)
    sc, P, u, v, w, run = case
    w = np.round(w * 2.0 ** 20) / 2.0 ** 20
    g = run(u, v, w)
    rng = np.random.default_rng(3)
    dirn = np.zeros_like(w)
    per = CN.param_count(1, C)
    for k in range(S):
        o = k * per + per - (C + 1)
        dirn[o:o + C + 1] = rng.choice([-1.0, 1.0], C + 1)
    gd = float(g["dp"] @ dirn)
    for h, tol in ((2.0 ** -10, 1e-3), (2.0 ** -3, 1e-5)):
        fd = (run(u, v, w + h * dirn, grads=False)["loss"] - run(u, v, w - h * dirn, grads=False)["loss"]) / (2 * h)
        say("head FD h", h, fd, "adjoint", gd)
        assert fd == pytest.approx(gd, rel=tol)
