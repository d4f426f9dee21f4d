"""Pins of the oracle's Unet adjoint (Sec. 3.1's Unet, Fig. 4, inside the
training loss of Sec. 3.2): the max-pooling and upsampling adjoints by
dot-product identities and against PyTorch's own backward, the whole
network forward and gradient against an independent PyTorch CPU rendering
differentiated by autograd (FP64), and the full loss gradient (network plus
Jacobi sweeps plus divergence) against central finite differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import scenes
from oracle import grid as G
from oracle import papernets as PN
from oracle import unet_adjoint as UA


def test_maxpool_adjoint_dot_product():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((8, 12, 5))
    v = rng.standard_normal(x.shape)
    w = rng.standard_normal((4, 6, 5))
    # the Jacobian of max pooling at x picks the value at each window's maximum
    ia, ib, ic, ie = UA.maxpool2_argmax(x)
    Jv = ia * v[0::2, 0::2] + ib * v[0::2, 1::2] + ic * v[1::2, 0::2] + ie * v[1::2, 1::2]
    assert np.isclose(np.sum(Jv * w), np.sum(v * UA.maxpool2_T(x, w)), rtol=1e-13)
    # and the masks select the maximum
    assert np.array_equal(ia * x[0::2, 0::2] + ib * x[0::2, 1::2] + ic * x[1::2, 0::2]
                          + ie * x[1::2, 1::2], PN.maxpool2(x))


def test_maxpool_adjoint_matches_torch_including_ties():
    rng = np.random.default_rng(1)
    x = rng.integers(0, 3, (8, 10, 4)).astype(np.float64)  # many ties
    w = rng.standard_normal((4, 5, 4))
    xt = torch.from_numpy(x).permute(2, 0, 1)[None].requires_grad_(True)
    y = F.max_pool2d(xt, 2)
    (y * torch.from_numpy(w).permute(2, 0, 1)[None]).sum().backward()
    ref = xt.grad[0].permute(1, 2, 0).numpy()
    assert np.array_equal(UA.maxpool2_T(x, w), ref)


def test_upsample_adjoint_dot_product():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((5, 7, 3))
    b = rng.standard_normal((10, 14, 3))
    assert np.isclose(np.sum(PN.up2c(a) * b), np.sum(a * UA.up2c_T(b)), rtol=1e-13)


def torch_unet(x, params):
    """The Unet written with PyTorch CPU modules (NCHW): replicate-padded
    3x3 convolutions with ReLU, 2x2 max pooling, bilinear x2 upsampling with
    half-pixel centres, skip channels first in the concatenation, a linear
    1x1 output."""
    o, layers = 0, []
    for (k, ci, co, relu) in PN.unet_layers():
        W = params[o:o + co * k * k * ci].reshape(co, k, k, ci).permute(0, 3, 1, 2); o += co * k * k * ci
        b = params[o:o + co]; o += co
        layers.append((W, b, relu, k))

    def conv(h, i):
        W, b, relu, k = layers[i]
        out = F.conv2d(F.pad(h, (k // 2,) * 4, mode="replicate"), W, b)
        return torch.relu(out) if relu else out

    h, li, skips = x, 0, []
    n = len(PN.UNET_WIDTHS)
    for lev in range(n):
        h = conv(conv(h, li), li + 1)
        li += 2
        if lev < n - 1:
            skips.append(h)
            h = F.max_pool2d(h, 2)
    for lev in range(n - 2, -1, -1):
        h = torch.cat([skips[lev], F.interpolate(h, scale_factor=2, mode="bilinear",
                                                 align_corners=False)], dim=1)
        h = conv(conv(h, li), li + 1)
        li += 2
    return conv(h, li)[0, 0]


def _case(n, seed, nobs=1):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    w = scenes.random_paper_weights("unet", seed).astype(np.float64)  # perturbed in FP64 below
    return sc, u, v, w


def test_unet_forward_and_gradient_match_torch_autograd():
    """With the Jacobi part removed (K = 0) the loss is a functional of the
    network output alone; its parameter gradient through the oracle's
    reverse pass must equal autograd through the PyTorch rendering."""
    n = 32
    sc, u, v, w = _case(n, 3)
    P = G.plan(sc.flags)
    ub, vb = G.enforce_bc(P, u, v)
    d = G.divergence(P, ub, vb, sc.dx)
    phi0, Fw = UA.unet_forward(P, d, sc.dx, w)
    s = Fw["s"]
    x = torch.from_numpy(np.stack([np.where(P.fluid, d / s, 0.0), (~P.fluid).astype(np.float64)]))[None]
    pt = torch.from_numpy(np.asarray(w, np.float64)).requires_grad_(True)
    y = torch_unet(x, pt)
    assert np.allclose(y.detach().numpy(), Fw["y"], rtol=0, atol=1e-11 * np.abs(Fw["y"]).max())
    # loss = sum_F r^2 with phi = phi0 (no sweeps): r = d - L phi0
    fl = torch.from_numpy(P.fluid)
    phi = torch.where(fl, sc.dx * sc.dx * s * y, torch.zeros_like(y))
    r = torch.from_numpy(d) - laplacian_t(P, phi, sc.dx)
    loss = (torch.where(fl, r, torch.zeros_like(r)) ** 2).sum()
    loss.backward()
    l_o, _, _, g_o = UA.loss_and_grad(sc.flags, u, v, sc.dx, w, K=0)
    assert l_o == pytest.approx(float(loss), rel=1e-12)
    ref = pt.grad.numpy()
    assert np.linalg.norm(g_o - ref) <= 1e-10 * np.linalg.norm(ref)


def laplacian_t(P, phi, dx):
    """The masked Laplacian of grid.laplacian on a torch tensor."""
    ny, nx = P.shape
    z = torch.zeros((ny + 2, nx + 2), dtype=phi.dtype)
    z[1:-1, 1:-1] = phi
    m = lambda a: torch.from_numpy(a.astype(np.float64))
    s = (m(P.nE) * (z[1:-1, 2:] - phi) + m(P.nW) * (z[1:-1, :-2] - phi)
         + m(P.nN) * (z[2:, 1:-1] - phi) + m(P.nS) * (z[:-2, 1:-1] - phi))
    return torch.where(torch.from_numpy(P.fluid), s / (dx * dx), torch.zeros_like(s))


def test_full_loss_gradient_matches_central_differences():
    """The whole chain (faces -> divergence -> normalisation -> Unet -> K
    Jacobi sweeps -> residual) against central differences in FP64, on a
    sample of parameters of every layer and of open faces."""
    n, K = 32, 4
    sc, u, v, w = _case(n, 4, nobs=2)
    P = G.plan(sc.flags)
    loss, gu, gv, gp = UA.loss_and_grad(sc.flags, u, v, sc.dx, w, K)
    rng = np.random.default_rng(5)
    offs, o = [], 0
    for (k, ci, co, _r) in PN.unet_layers():
        offs.append(o)
        o += k * k * ci * co + co
    picks = [int(off + rng.integers(0, (k * k * ci * co + co)))
             for off, (k, ci, co, _r) in zip(offs, PN.unet_layers())]
    for i in picks:
        h = 1e-5 * max(1.0, abs(w[i]))
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (UA.loss_only(sc.flags, u, v, sc.dx, wp, K) - UA.loss_only(sc.flags, u, v, sc.dx, wm, K)) / (2 * h)
        assert gp[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss)), i
    ju, iu = np.nonzero(P.uopen)
    for q in rng.choice(len(ju), 6, replace=False):
        h = 1e-6
        up_, um = u.copy(), u.copy()
        up_[ju[q], iu[q]] += h
        um[ju[q], iu[q]] -= h
        fd = (UA.loss_only(sc.flags, up_, v, sc.dx, w, K) - UA.loss_only(sc.flags, um, v, sc.dx, w, K)) / (2 * h)
        assert gu[ju[q], iu[q]] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))
