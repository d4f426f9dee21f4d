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
