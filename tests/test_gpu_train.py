"""Solver-in-the-loop training on the GPU (library forward, adjoint and Adam
kernels) and the gain test: the trained network must leave less divergence
after its guess and need fewer Jacobi sweeps than the method without it."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from paper_2109_09363_amd import train as TR

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def held_out_states(n, count=4, seed=4242):
    """u* of a plume that the plain solver advances (not in the training set)."""
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=2)
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0)
    tf = torch.from_numpy(sc.flags).cuda()
    pr.plan(tf)
    rho = torch.full((n, n), sc.rho0, dtype=torch.float32, device="cuda")
    u = torch.zeros((n, n + 1), dtype=torch.float32, device="cuda")
    v = torch.zeros((n + 1, n), dtype=torch.float32, device="cuda")
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    out = []
    for s in range(6 + 3 * count):
        xi = torch.from_numpy(scenes.inflow_noise(seed, s, n).astype(np.float32)).cuda()
        pr.advect_async(rho, u, v, xi, g=sc.g, drho=sc.drho, u_in=sc.u_in)
        if s >= 6 and (s - 6) % 3 == 0:
            out.append((tf, u.clone(), v.clone()))
        pr.project_async(u, v, tf, p, 1e-3, method="pcg", max_iters=20000)
    torch.cuda.synchronize()
    return sc, out


def sweeps_to_threshold(n, S, C, w, states, rel=0.05):
    pr = hp.Projector(n, n, 1.0 / n, 1.0, 1.0, S, C, "fp32")
    tw = torch.from_numpy(w.astype(np.float32)).cuda()
    pr.set_weights(tw)
    p = torch.empty((n, n), dtype=torch.float32, device="cuda")
    iters, e_cnn = [], []
    for tf, u, v in states:
        pr.plan(tf)
        uu, vv = u.clone(), v.clone()
        pr.project_async(uu, vv, tf, p, 0.0, method="cnn")
        r0 = pr.result()
        thr = rel * r0.e1_init
        uu, vv = u.clone(), v.clone()
        pr.project_async(uu, vv, tf, p, thr, method="hybrid", max_iters=200000, check_every=4)
        r = pr.result()
        assert r.status == 0
        iters.append(r.iters)
        e_cnn.append(r.e1_cnn / r.e1_init)
    return np.array(iters), np.array(e_cnn)


def test_training_gain():
    n, S, C = 64, 3, 16
    torch.manual_seed(0)
    data = TR.generate_dataset(n, n_scenes=6, steps=20, keep_every=2, n_random=24, seed=3, log=say)
    w0 = scenes.random_weights(S, C, 1, out_scale=0.1)
    w, hist = TR.train(data, n, S, C, "fp32", steps=300, batch=4, lr=2e-3, sweeps=4, params0=w0,
                       seed=1, log=say, log_every=50)
    say("loss history", hist)
    assert hist[-1][1] < 0.5 * hist[0][1]
    sc, states = held_out_states(n)
    zero = w.copy()
    per = (C * 18 + C) + 3 * (C * 9 * C + C) + C + 1
    for k in range(S):  # zero output layer: the guess is 0 -> plain Jacobi
        zero[k * per + per - (C + 1): (k + 1) * per] = 0.0
    it_t, e_t = sweeps_to_threshold(n, S, C, w, states)
    it_z, e_z = sweeps_to_threshold(n, S, C, zero, states)
    say("held-out sweeps trained", it_t, "untrained", it_z)
    say("held-out E1 after guess / E1 init: trained", e_t, "zero", e_z)
    assert np.all(e_t < e_z)
    assert it_t.sum() < it_z.sum()


@pytest.mark.parametrize("n,S,C,K,n_unroll,seed", [(32, 2, 16, 2, 4, 0), (48, 3, 16, 4, 16, 1)])
def test_long_term_gradient_matches_oracle(n, S, C, K, n_unroll, seed):
    """Short-term + long-term loss gradient (unrolled plume steps through the
    library's advection and projection, only the last projection
    differentiated) against the FP64 oracle's own unrolled run."""
    from oracle import adjoint as AJ
    from tests.gpu_util import to_dev, f32, rel_l2
    say("long-term", n, S, C, K, n_unroll, seed)
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1, ri=0.1)
    u, v = (f32(a) for a in scenes.random_faces(n, n, seed, kind="smooth"))
    rho = f32(scenes.random_density(n, n, seed, sc.rho0, sc.drho))
    w = f32(scenes.random_weights(S, C, seed))
    xis = [f32(scenes.inflow_noise(seed, j, n)) for j in range(n_unroll)]
    alpha, beta = 0.7, 1.3
    o = AJ.long_term(sc.flags, rho, u, v, sc.dx, w, S, C, K, n_unroll, alpha, beta, sc.g, sc.rho0,
                     sc.drho, sc.u_in, xis)
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0, S, C, "fp32", train=True)
    pr.set_weights(to_dev(w))
    tf = to_dev(sc.flags, torch.uint8)
    smp = TR.Sample(tf, to_dev(u), to_dev(v), to_dev(rho), sc.g, sc.drho, sc.u_in, seed)
    p = torch.empty((n, n), dtype=torch.float32, device="cuda")
    pr.plan(tf)
    pr.project_async(smp.u.clone(), smp.v.clone(), tf, p, 0.0, method="cnn")
    r = pr.result()
    norm_short = 1.0 / (r.s * r.s * r.n_fluid)
    grads = torch.zeros(pr.param_count, dtype=torch.float32, device="cuda")
    ls = torch.zeros(1, dtype=torch.float64, device="cuda")
    ll = torch.zeros(1, dtype=torch.float64, device="cuda")
    TR.unrolled_backward(pr, smp, K, n_unroll, alpha, beta, norm_short, grads,
                         [to_dev(x) for x in xis], loss_short=ls, loss_long=ll)
    torch.cuda.synchronize()
    gp = grads.cpu().numpy().astype(np.float64)
    err = rel_l2(gp, o["dparams"])
    say("  loss short gpu", float(ls.item()), "oracle", o["loss_short"], "long gpu", float(ll.item()),
        "oracle", o["loss_long"], "rel L2 dparams", err)
    assert float(ls.item()) == pytest.approx(o["loss_short"], rel=1e-5)
    assert float(ll.item()) == pytest.approx(o["loss_long"], rel=1e-3)
    assert err <= 1e-3
    # the sample itself is left untouched
    assert np.array_equal(smp.u.cpu().numpy(), np.float32(u))


def test_long_term_training_runs():
    n, S, C = 32, 2, 16
    data = TR.generate_dataset(n, n_scenes=2, steps=6, keep_every=2, n_random=4, seed=5, log=say)
    w, hist = TR.train(data, n, S, C, "fp32", steps=6, batch=2, lr=1e-3, sweeps=2, seed=2,
                       log=say, log_every=2, alpha=1.0, beta=1.0)
    assert np.all(np.isfinite(w)) and all(np.isfinite(h[1]) and h[1] > 0 for h in hist)
