"""Pins of the oracle's cascade adjoint (Sec. 3.1's MultiScale / SmallScale,
Fig. 3, inside the training loss of Sec. 3.2): the k x k convolution adjoint
(k = 1, 3, 5) against PyTorch's own backward of a replicate-padded conv2d,
the down-sampling adjoint by a dot-product identity and against PyTorch's
bilinear interpolation backward, the whole cascade's parameter gradient
against autograd through an independent PyTorch rendering (FP64), and the
full loss gradient (network plus Jacobi sweeps plus divergence) against
central differences."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import scenes
from oracle import cascade_adjoint as CA
from oracle import grid as G
from oracle import papernets as PN


@pytest.mark.parametrize("k,cin,cout", [(1, 6, 1), (3, 4, 5), (5, 3, 4)])
def test_convk_backward_matches_torch(k, cin, cout):
    rng = np.random.default_rng(k)
    x = rng.standard_normal((9, 11, cin))
    W = rng.standard_normal((cout, k, k, cin))
    b = rng.standard_normal(cout)
    lam = rng.standard_normal((9, 11, cout))
    lx, dW, db = CA.convk_backward(x, W, lam)
    xt = torch.from_numpy(x).permute(2, 0, 1)[None].requires_grad_(True)
    Wt = torch.from_numpy(W).permute(0, 3, 1, 2).contiguous().requires_grad_(True)
    bt = torch.from_numpy(b).requires_grad_(True)
    out = F.conv2d(F.pad(xt, (k // 2,) * 4, mode="replicate") if k > 1 else xt, Wt, bt)
    assert np.allclose(out[0].permute(1, 2, 0).detach().numpy(), PN.conv_replicate(x, W, b), atol=1e-12)
    (out * torch.from_numpy(lam).permute(2, 0, 1)[None]).sum().backward()
    assert np.allclose(lx, xt.grad[0].permute(1, 2, 0).numpy(), atol=1e-11)
    assert np.allclose(dW, Wt.grad.permute(0, 2, 3, 1).numpy(), atol=1e-10)
    assert np.allclose(db, bt.grad.numpy(), atol=1e-11)


@pytest.mark.parametrize("f", [2, 4])
def test_down_adjoint(f):
    rng = np.random.default_rng(f)
    x = rng.standard_normal((16, 24, 1))
    lam = rng.standard_normal((16 // f, 24 // f))
    assert np.isclose(np.sum(PN.down(x, f)[:, :, 0] * lam), np.sum(x[:, :, 0] * CA.down_T(lam, f, (16, 24))),
                      rtol=1e-13)
    xt = torch.from_numpy(x[:, :, 0])[None, None].requires_grad_(True)
    y = F.interpolate(xt, scale_factor=1.0 / f, mode="bilinear", align_corners=False)
    (y * torch.from_numpy(lam)[None, None]).sum().backward()
    assert np.allclose(CA.down_T(lam, f, (16, 24)), xt.grad[0, 0].numpy(), atol=1e-13)


def torch_cascade_phi0(d, fluid, dx, p, arch):
    """phi0 of the cascade written with PyTorch CPU modules (parameters a
    torch tensor, so that autograd differentiates it)."""
    s = float(np.sqrt(np.sum(d[fluid] ** 2) / fluid.sum()))
    x = torch.from_numpy(np.stack([np.where(fluid, d / s, 0.0), (~fluid).astype(np.float64)]))[None]
    ins = [F.interpolate(x, scale_factor=0.25, mode="bilinear", align_corners=False),
           F.interpolate(x, scale_factor=0.5, mode="bilinear", align_corners=False), x]
    o, y = 0, None
    for b, layers in enumerate(PN.branches(arch)):
        h = ins[b]
        if y is not None:
            h = torch.cat([h, F.interpolate(y, scale_factor=2, mode="bilinear", align_corners=False)], dim=1)
        for i, (k, ci, co, _relu) in enumerate(layers):
            W = p[o:o + co * k * k * ci].reshape(co, k, k, ci).permute(0, 3, 1, 2); o += co * k * k * ci
            bias = p[o:o + co]; o += co
            h = F.conv2d(F.pad(h, (k // 2,) * 4, mode="replicate") if k > 1 else h, W, bias)
            if i < len(layers) - 2:
                h = torch.relu(h)
        y = h
    fl = torch.from_numpy(fluid)
    return torch.where(fl, dx * dx * s * y[0, 0], torch.zeros_like(y[0, 0])), s


def _case(arch, n, seed, nobs=1):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    w = scenes.random_paper_weights(arch, seed).astype(np.float64)
    return sc, u, v, w


@pytest.mark.parametrize("arch,n,seed", [("smallscale", 32, 3), ("multiscale", 16, 4)])
def test_cascade_gradient_matches_torch_autograd(arch, n, seed):
    """With no Jacobi sweeps (K = 0) the loss is a functional of the
    network output; its parameter gradient through the oracle's reverse
    pass must equal autograd through the PyTorch rendering."""
    sc, u, v, w = _case(arch, n, seed)
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    pt = torch.from_numpy(w).requires_grad_(True)
    phi, _s = torch_cascade_phi0(d, P.fluid, sc.dx, pt, arch)
    phi_o, _F = CA.cascade_forward(P, d, sc.dx, w, arch)
    assert np.allclose(phi.detach().numpy(), phi_o, rtol=0, atol=1e-11 * np.abs(phi_o).max())
    from tests.test_oracle_unet_adjoint import laplacian_t
    r = torch.from_numpy(d) - laplacian_t(P, phi, sc.dx)
    loss = (torch.where(torch.from_numpy(P.fluid), r, torch.zeros_like(r)) ** 2).sum()
    loss.backward()
    l_o, _, _, g_o = CA.loss_and_grad(sc.flags, u, v, sc.dx, w, arch, K=0)
    assert l_o == pytest.approx(float(loss.detach()), rel=1e-12)
    ref = pt.grad.numpy()
    assert np.linalg.norm(g_o - ref) <= 1e-10 * np.linalg.norm(ref)


def test_cascade_full_loss_gradient_matches_central_differences():
    """The whole chain (faces -> divergence -> normalisation -> cascade -> K
    Jacobi sweeps -> residual) against central differences in FP64, on a
    sample of parameters of every layer of every branch and of open faces."""
    arch, n, K = "smallscale", 32, 4
    sc, u, v, w = _case(arch, n, 6, nobs=2)
    P = G.plan(sc.flags)
    loss, gu, gv, gp = CA.loss_and_grad(sc.flags, u, v, sc.dx, w, arch, K)
    rng = np.random.default_rng(7)
    o, picks = 0, []
    for br in PN.branches(arch):
        for (k, ci, co, _r) in br:
            m = k * k * ci * co + co
            picks.append(int(o + rng.integers(0, m)))
            o += m
    for i in picks:
        h = 1e-5 * max(1.0, abs(w[i]))
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (CA.loss_only(sc.flags, u, v, sc.dx, wp, arch, K) - CA.loss_only(sc.flags, u, v, sc.dx, wm, arch, K)) / (2 * h)
        assert gp[i] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss)), i
    ju, iu = np.nonzero(P.uopen)
    for q in rng.choice(len(ju), 5, replace=False):
        h = 1e-6
        up_, um = u.copy(), u.copy()
        up_[ju[q], iu[q]] += h
        um[ju[q], iu[q]] -= h
        fd = (CA.loss_only(sc.flags, up_, v, sc.dx, w, arch, K) - CA.loss_only(sc.flags, um, v, sc.dx, w, arch, K)) / (2 * h)
        assert gu[ju[q], iu[q]] == pytest.approx(fd, rel=1e-5, abs=1e-9 * abs(loss))


def test_cascade_adjoint_detects_a_wrong_coarse_path():
    """A planted mistake in the oracle (the coarse output's gradient taken by
    sub-sampling the fine one instead of the transposed bilinear x2) must
    fail the autograd comparison: the test above sees the coarse path."""
    arch, n, seed = "smallscale", 32, 3
    sc, u, v, w = _case(arch, n, seed)
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    pt = torch.from_numpy(w).requires_grad_(True)
    phi, _s = torch_cascade_phi0(d, P.fluid, sc.dx, pt, arch)
    from tests.test_oracle_unet_adjoint import laplacian_t
    r = torch.from_numpy(d) - laplacian_t(P, phi, sc.dx)
    (torch.where(torch.from_numpy(P.fluid), r, torch.zeros_like(r)) ** 2).sum().backward()
    good = CA.up2_T
    try:
        CA.up2_T = lambda lam: 4.0 * lam[0::2, 0::2]
        _, _, _, g_bad = CA.loss_and_grad(sc.flags, u, v, sc.dx, w, arch, K=0)
    finally:
        CA.up2_T = good
    ref = pt.grad.numpy()
    assert np.linalg.norm(g_bad - ref) > 1e-3 * np.linalg.norm(ref)
