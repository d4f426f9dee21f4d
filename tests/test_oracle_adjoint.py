"""Pins of the oracle adjoint (gradient of the divergence loss through the
CNN guess and K Jacobi sweeps): central finite differences in FP64 and
dot-product (transpose) identities of the linear stages.

The loss is piecewise smooth (ReLU kinks), so the FD step is h = 1e-6 here;
a step of 1e-3 moves some pre-activations across zero, and the h = 1e-3 test
below only uses parameters whose ReLU pattern is the same at both points."""
import numpy as np
import pytest

import scenes
from oracle import adjoint as AJ
from oracle import advect as AD
from oracle import cnn as CN
from oracle import grid as G


def setup(n=16, S=2, C=4, seed=0, nobs=1):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    w = scenes.random_weights(S, C, seed).astype(np.float64)
    return sc, u, v, w


def fd(f, x, idx, h=1e-6):
    xp = x.copy(); xm = x.copy()
    xp.flat[idx] += h; xm.flat[idx] -= h
    return (f(xp) - f(xm)) / (2 * h)


@pytest.mark.parametrize("K,omega", [(0, 1.0), (3, 1.0), (5, 0.8)])
def test_grad_params_fd(K, omega):
    sc, u, v, w = setup(seed=1)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 2, 4, K, omega)
    f = lambda ww: AJ.loss_and_grad(sc.flags, u, v, sc.dx, ww, 2, 4, K, omega)[0]
    rng = np.random.default_rng(0)
    idx = rng.choice(w.size, 25, replace=False)
    num = np.array([fd(f, w, i) for i in idx])
    assert np.allclose(gp[idx], num, rtol=1e-5, atol=1e-8 * np.abs(gp).max())
    # directional derivative along a random direction
    dirn = rng.standard_normal(w.size)
    dd = (f(w + 1e-6 * dirn) - f(w - 1e-6 * dirn)) / 2e-6
    assert dd == pytest.approx(float(gp @ dirn), rel=1e-5)


def relu_pattern(sc, u, v, w, S, C):
    P = G.plan(sc.flags)
    _, F = AJ.forward(P, u, v, sc.dx, w, S, C, 0)
    return np.concatenate([(a > 0).ravel() for acts in F["cache"]["acts"] for a in acts[1:]])


def test_grad_params_fd_h1e3_kink_free():
    sc, u, v, w = setup(seed=1)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 2, 4, 3)
    f = lambda ww: AJ.loss_and_grad(sc.flags, u, v, sc.dx, ww, 2, 4, 3)[0]
    base = relu_pattern(sc, u, v, w, 2, 4)
    rng = np.random.default_rng(5)
    used = 0
    for i in rng.choice(w.size, 60, replace=False):
        wp = w.copy(); wp[i] += 1e-3
        wm = w.copy(); wm[i] -= 1e-3
        if not (np.array_equal(relu_pattern(sc, u, v, wp, 2, 4), base) and
                np.array_equal(relu_pattern(sc, u, v, wm, 2, 4), base)):
            continue
        used += 1
        num = (f(wp) - f(wm)) / 2e-3
        assert gp[i] == pytest.approx(num, rel=1e-6, abs=1e-9 * np.abs(gp).max())
    assert used >= 20


@pytest.mark.parametrize("K", [0, 4])
def test_grad_velocity_fd(K):
    sc, u, v, w = setup(seed=2)
    P = G.plan(sc.flags)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 2, 4, K)
    fu = lambda uu: AJ.loss_and_grad(sc.flags, uu, v, sc.dx, w, 2, 4, K)[0]
    fv = lambda vv: AJ.loss_and_grad(sc.flags, u, vv, sc.dx, w, 2, 4, K)[0]
    rng = np.random.default_rng(1)
    for idx in rng.choice(u.size, 12, replace=False):
        assert gu.flat[idx] == pytest.approx(fd(fu, u, idx), rel=1e-5, abs=1e-7 * np.abs(gu).max())
    # include inflow faces and top faces
    cand = list(rng.choice(v.size, 10, replace=False)) + [int(np.nonzero(P.vinflow)[0][0]),
                                                          v.size - 3]
    for idx in cand:
        assert gv.flat[idx] == pytest.approx(fd(fv, v, idx), rel=1e-5, abs=1e-7 * np.abs(gv).max())
    assert np.all(gu[~P.uopen] == 0)


def test_grad_three_scales_fd():
    sc, u, v, w = setup(n=16, S=3, C=3, seed=3, nobs=2)
    loss, gu, gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 3, 3, 2)
    rng = np.random.default_rng(2)
    f = lambda ww: AJ.loss_and_grad(sc.flags, u, v, sc.dx, ww, 3, 3, 2)[0]
    dirn = rng.standard_normal(w.size)
    dd = (f(w + 1e-6 * dirn) - f(w - 1e-6 * dirn)) / 2e-6
    assert dd == pytest.approx(float(gp @ dirn), rel=1e-5)
    fu = lambda uu: AJ.loss_and_grad(sc.flags, uu, v, sc.dx, w, 3, 3, 2)[0]
    du = rng.standard_normal(u.shape)
    dd = (fu(u + 1e-6 * du) - fu(u - 1e-6 * du)) / 2e-6
    assert dd == pytest.approx(float(np.sum(gu * du)), rel=1e-5)


def test_dot_product_up2_and_down2():
    rng = np.random.default_rng(3)
    t = rng.standard_normal((5, 7))
    lam = rng.standard_normal((10, 14))
    assert np.sum(CN.up2(t) * lam) == pytest.approx(np.sum(t * AJ.up2_T(lam)), rel=1e-13)
    x = rng.standard_normal((8, 6))
    y = rng.standard_normal((4, 3))
    assert np.sum(CN.down2(x[:, :, None])[:, :, 0] * y) == pytest.approx(
        np.sum(x * AJ.down2_T(y)), rel=1e-13)


def test_dot_product_conv_input():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((6, 5, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = np.zeros(4)
    lam = rng.standard_normal((6, 5, 4))
    lx, dW, db = AJ.conv3x3_backward(x, W, lam)
    assert np.sum(CN.conv3x3_replicate(x, W, b) * lam) == pytest.approx(np.sum(x * lx), rel=1e-12)
    assert np.sum(CN.conv3x3_replicate(x, W, b) * lam) == pytest.approx(np.sum(W * dW), rel=1e-12)


def lt_setup(n=16, S=2, C=4, seed=3):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1, ri=0.1)
    u, v = scenes.random_faces(n, n, seed, kind="smooth")
    rho = scenes.random_density(n, n, seed, sc.rho0, sc.drho)
    w = scenes.random_weights(S, C, seed).astype(np.float64)
    xis = [scenes.inflow_noise(seed, j, n) for j in range(4)]
    return sc, rho, u, v, w, xis


def lt(sc, rho, u, v, w, xis, n, alpha, beta, K=2):
    return AJ.long_term(sc.flags, rho, u, v, sc.dx, w, 2, 4, K, n, alpha, beta, sc.g, sc.rho0,
                        sc.drho, sc.u_in, xis)


def test_long_term_weights_are_linear():
    sc, rho, u, v, w, xis = lt_setup()
    a = lt(sc, rho, u, v, w, xis, 3, 1.0, 0.0)
    b = lt(sc, rho, u, v, w, xis, 3, 0.0, 1.0)
    c = lt(sc, rho, u, v, w, xis, 3, 2.0, 3.0)
    assert a["loss_long"] == 0.0 and b["loss_short"] == 0.0
    assert c["loss"] == pytest.approx(2 * a["loss"] + 3 * b["loss"], rel=1e-12)
    assert np.allclose(c["dparams"], 2 * a["dparams"] + 3 * b["dparams"], rtol=1e-12, atol=1e-15)
    # the short term alone is the single-projection loss, normalised by sum_F d^2
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    l0, _, _, g0 = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 2, 4, 2)
    nrm = float(np.sum(d[P.fluid] ** 2))
    assert a["loss"] == pytest.approx(l0 / nrm, rel=1e-12)
    assert np.allclose(a["dparams"], g0 / nrm, rtol=1e-12, atol=1e-15)


def test_long_term_rollout_starts_from_corrected_velocity():
    # The loss of the short term is the divergence energy of the corrected
    # velocity (computed here from the faces), which is what the first
    # unrolled advection must receive.
    sc, rho, u, v, w, xis = lt_setup(seed=4)
    P = G.plan(sc.flags)
    uc, vc = AJ.hybrid_corrected(P, u, v, sc.dx, w, 2, 4, 2)
    dc = G.divergence(P, uc, vc, sc.dx)
    l0 = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, 2, 4, 2)[0]
    assert float(np.sum(dc[P.fluid] ** 2)) == pytest.approx(l0, rel=1e-9)
    one = lt(sc, rho, u, v, w, xis, 1, 1.0, 1.0)
    dt = AD.cfl_dt(uc, vc, sc.dx, sc.u_in)
    r1, us, vs = AD.advect_step(P, sc.flags, rho, uc, vc, sc.dx, dt, sc.g, sc.rho0, sc.drho,
                                sc.u_in, xis[0])
    assert np.array_equal(one["u_star"], us) and np.array_equal(one["v_star"], vs)
    assert np.array_equal(one["rho"], r1)


def test_long_term_two_steps_compose():
    # n = 2 is n = 1, the frozen network's correction of u*_{t+1}, and one
    # more step with the second inflow perturbation.
    sc, rho, u, v, w, xis = lt_setup(seed=5)
    P = G.plan(sc.flags)
    one = lt(sc, rho, u, v, w, xis, 1, 1.0, 1.0)
    two = lt(sc, rho, u, v, w, xis, 2, 1.0, 1.0)
    uc, vc = AJ.hybrid_corrected(P, one["u_star"], one["v_star"], sc.dx, w, 2, 4, 2)
    dt = AD.cfl_dt(uc, vc, sc.dx, sc.u_in)
    r2, us, vs = AD.advect_step(P, sc.flags, one["rho"], uc, vc, sc.dx, dt, sc.g, sc.rho0,
                                sc.drho, sc.u_in, xis[1])
    assert np.array_equal(two["u_star"], us) and np.array_equal(two["v_star"], vs)
    assert np.array_equal(two["rho"], r2)
    assert two["loss_short"] == one["loss_short"]
    assert not np.array_equal(two["u_star"], one["u_star"])


def test_long_term_gradient_is_frozen_state_derivative():
    # Advection is not differentiated: the long-term gradient is the
    # derivative of the last projection's loss with the unrolled state held
    # fixed (central differences in FP64 along random directions).
    sc, rho, u, v, w, xis = lt_setup(seed=6)
    b = lt(sc, rho, u, v, w, xis, 3, 0.0, 1.0)
    P = G.plan(sc.flags)
    us, vs = b["u_star"], b["v_star"]
    d = G.divergence(P, *G.enforce_bc(P, us, vs), sc.dx)
    scale = 1.0 / float(np.sum(d[P.fluid] ** 2))
    f = lambda ww: AJ.forward(P, us, vs, sc.dx, ww, 2, 4, 2, 1.0, scale)[0]
    assert f(w) == pytest.approx(b["loss"], rel=1e-12)
    rng = np.random.default_rng(7)
    for _ in range(3):
        dirn = rng.standard_normal(w.size)
        dd = (f(w + 1e-6 * dirn) - f(w - 1e-6 * dirn)) / 2e-6
        assert dd == pytest.approx(float(b["dparams"] @ dirn), rel=1e-5)


def test_bf16_emulated_loss_is_the_projection_with_the_bf16_network():
    """The loss of loss_and_grad(bf16=True) is the divergence energy left by
    the hybrid projection with the BF16-emulated network and K sweeps (the
    forward of project.project, an independent path); its gradient is the
    straight-through reading (rounded activations, unrounded weights), which
    no finite difference can check since a rounding is piecewise constant."""
    from oracle import project as PR
    n, S, C, K = 32, 3, 16, 5
    sc = scenes.plume_scene(n, seed=8, n_obstacles=2)
    u, v = scenes.random_faces(n, n, 8, kind="mixed")
    w = scenes.random_weights(S, C, 8).astype(np.float32).astype(np.float64)
    loss, _gu, _gv, gp = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K, bf16=True)
    o = PR.project(sc.flags, u, v, sc.dx, method="hybrid", params=w, S=S, C=C, bf16=True, fixed_iters=K)
    P = G.plan(sc.flags)
    r = G.divergence(P, o["u"], o["v"], sc.dx)
    assert loss == pytest.approx(float(np.sum(r[P.fluid] ** 2)), rel=1e-12)
    loss64, _a, _b, gp64 = AJ.loss_and_grad(sc.flags, u, v, sc.dx, w, S, C, K)
    assert loss != loss64 and np.linalg.norm(gp - gp64) < 0.2 * np.linalg.norm(gp64)
