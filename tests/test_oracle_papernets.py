"""Pins of the oracle's cascaded MultiScale / SmallScale networks (Sec. 3.1,
Fig. 3): parameter totals against the paper's, the resampling and the
convolutions against PyTorch's CPU routines, and the whole cascade against an
independent PyTorch CPU rendering of the same reading of the paper."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

import scenes
from oracle import cnn as CN
from oracle import grid as G
from oracle import papernets as PN


def test_parameter_totals_match_the_paper():
    # Fig. 3 caption: 418,640; SmallScale about 1.3e5 (Sec. 3.1)
    assert PN.param_count("multiscale") == 419459
    assert abs(PN.param_count("multiscale") - 418640) / 418640 < 0.003
    assert PN.param_count("smallscale") == 126819
    assert abs(PN.param_count("smallscale") - 1.3e5) / 1.3e5 < 0.03
    for arch in PN.ARCHS:
        br = PN.branches(arch)
        assert [len(b) for b in br] == [5, 7, 7]  # layers per scale (Sec. 3.1)
        for b in br:
            assert b[0][0] == 5 and b[-1][0] == 1 and b[-1][2] == 1
            assert [r for (_k, _ci, _co, r) in b[-2:]] == [False, False]
            assert all(r for (_k, _ci, _co, r) in b[:-2])
        assert br[0][0][1] == 2 and br[1][0][1] == 3 and br[2][0][1] == 3


@pytest.mark.parametrize("f", [2, 4])
def test_down_is_bilinear_half_pixel(f):
    rng = np.random.default_rng(f)
    x = rng.standard_normal((16, 24, 3))
    ref = F.interpolate(torch.from_numpy(x).permute(2, 0, 1)[None], scale_factor=1.0 / f,
                        mode="bilinear", align_corners=False)[0].permute(1, 2, 0).numpy()
    assert np.allclose(PN.down(x, f), ref, rtol=0, atol=1e-14)
    if f == 2:
        assert np.allclose(PN.down(x, 2), CN.down2(x), rtol=0, atol=1e-15)
    else:  # the mean of the central 2x2 pixels of every 4x4 block
        c = 0.25 * (x[1::4, 1::4] + x[2::4, 1::4] + x[1::4, 2::4] + x[2::4, 2::4])
        assert np.allclose(PN.down(x, 4), c, rtol=0, atol=1e-15)


@pytest.mark.parametrize("k", [1, 3, 5])
def test_conv_replicate_matches_torch(k):
    rng = np.random.default_rng(k)
    x = rng.standard_normal((9, 13, 3))
    W = rng.standard_normal((5, k, k, 3))
    b = rng.standard_normal(5)
    xt = F.pad(torch.from_numpy(x).permute(2, 0, 1)[None], (k // 2,) * 4, mode="replicate")
    ref = F.conv2d(xt, torch.from_numpy(W).permute(0, 3, 1, 2), torch.from_numpy(b))
    assert np.allclose(PN.conv_replicate(x, W, b), ref[0].permute(1, 2, 0).numpy(), atol=1e-12)


def torch_cascade(d, solid, fluid, dx, params, arch):
    """The paper's MultiScale written with PyTorch CPU modules: quarter and
    half-resolution copies of the input, coarse output upsampled x2 and
    concatenated as an extra input channel, ReLU on all but the last two
    layers of a branch."""
    s = float(np.sqrt(np.sum(d[fluid] ** 2) / fluid.sum()))
    x = torch.from_numpy(np.stack([np.where(fluid, d / s, 0.0), solid.astype(np.float64)]))[None]
    ins = [F.interpolate(x, scale_factor=0.25, mode="bilinear", align_corners=False),
           F.interpolate(x, scale_factor=0.5, mode="bilinear", align_corners=False), x]
    p = torch.from_numpy(np.asarray(params, np.float64))
    o, y = 0, None
    for b, layers in enumerate(PN.branches(arch)):
        h = ins[b]
        if y is not None:
            h = torch.cat([h, F.interpolate(y, scale_factor=2, mode="bilinear",
                                            align_corners=False)], dim=1)
        for i, (k, ci, co, _relu) in enumerate(layers):
            W = p[o:o + co * k * k * ci].reshape(co, k, k, ci).permute(0, 3, 1, 2); o += co * k * k * ci
            bias = p[o:o + co]; o += co
            h = F.conv2d(F.pad(h, (k // 2,) * 4, mode="replicate"), W, bias)
            if i < len(layers) - 2:
                h = torch.relu(h)
        y = h
    return np.where(fluid, dx * dx * s * y[0, 0].numpy(), 0.0)


@pytest.mark.parametrize("arch,n,seed", [("multiscale", 32, 0), ("smallscale", 48, 1),
                                          ("multiscale", 24, 2)])
def test_cascade_matches_torch_rendering(arch, n, seed):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1)
    P = G.plan(sc.flags)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    w = scenes.random_paper_weights(arch, seed)
    phi, s, ys = PN.phi0(P, d, sc.dx, w, arch)
    ref = torch_cascade(d, ~P.fluid, P.fluid, sc.dx, w, arch)
    assert np.abs(phi).max() > 0
    assert np.allclose(phi, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    assert [y.shape for y in ys] == [(n // 4, n // 4), (n // 2, n // 2), (n, n)]


def test_scale_invariance_and_solids():
    # phi0 is linear in the scale of d (the input is normalised by s)
    n = 32
    sc = scenes.plume_scene(n, seed=3, n_obstacles=2)
    P = G.plan(sc.flags)
    u, v = scenes.random_faces(n, n, 3, kind="smooth")
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    w = scenes.random_paper_weights("smallscale", 3)
    a = PN.phi0(P, d, sc.dx, w, "smallscale")[0]
    b = PN.phi0(P, 7.0 * d, sc.dx, w, "smallscale")[0]
    assert np.allclose(b, 7.0 * a, rtol=1e-12, atol=1e-15)
    assert np.all(a[~P.fluid] == 0.0)
    assert PN.phi0(P, np.zeros_like(d), sc.dx, w, "smallscale")[1] == 0.0


def test_unet_parameter_total_and_pooling():
    # Fig. 4 caption: 443,521 parameters
    assert PN.param_count("unet") == 443441
    assert abs(PN.param_count("unet") - 443521) / 443521 < 3e-4
    assert scenes.random_paper_weights("unet", 0).size == 443441
    rng = np.random.default_rng(9)
    x = rng.standard_normal((12, 20, 5))
    ref = F.max_pool2d(torch.from_numpy(x).permute(2, 0, 1)[None], 2)[0].permute(1, 2, 0).numpy()
    assert np.array_equal(PN.maxpool2(x), ref)
    ref = F.interpolate(torch.from_numpy(x).permute(2, 0, 1)[None], scale_factor=2, mode="bilinear",
                        align_corners=False)[0].permute(1, 2, 0).numpy()
    assert np.allclose(PN.up2c(x), ref, rtol=0, atol=1e-14)


def torch_unet(d, solid, fluid, dx, params):
    """The Unet of Sec. 3.1 with PyTorch CPU modules: two 3x3 + ReLU per
    scale, max pooling down, bilinear x2 up, skip concatenated before the
    upsampled map, linear 1x1 output."""
    s = float(np.sqrt(np.sum(d[fluid] ** 2) / fluid.sum()))
    h = torch.from_numpy(np.stack([np.where(fluid, d / s, 0.0), solid.astype(np.float64)]))[None]
    p = torch.from_numpy(np.asarray(params, np.float64))
    shapes = scenes.paper_net_layers("unet")[0]
    o = [0]

    def layer(h, i, relu=True):
        k, ci, co = shapes[i]
        W = p[o[0]:o[0] + co * k * k * ci].reshape(co, k, k, ci).permute(0, 3, 1, 2)
        o[0] += co * k * k * ci
        b = p[o[0]:o[0] + co]
        o[0] += co
        out = F.conv2d(F.pad(h, (k // 2,) * 4, mode="replicate"), W, b)
        return torch.relu(out) if relu else out

    skips, i = [], 0
    for lev in range(5):
        h = layer(layer(h, i), i + 1)
        i += 2
        if lev < 4:
            skips.append(h)
            h = F.max_pool2d(h, 2)
    for lev in range(3, -1, -1):
        up = F.interpolate(h, scale_factor=2, mode="bilinear", align_corners=False)
        h = torch.cat([skips[lev], up], dim=1)
        h = layer(layer(h, i), i + 1)
        i += 2
    y = layer(h, i, relu=False)
    assert o[0] == p.numel()
    return np.where(fluid, dx * dx * s * y[0, 0].numpy(), 0.0)


@pytest.mark.parametrize("n,seed", [(32, 0), (48, 1)])
def test_unet_matches_torch_rendering(n, seed):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=1)
    P = G.plan(sc.flags)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    w = scenes.random_paper_weights("unet", seed)
    phi, s = PN.unet_phi0(P, d, sc.dx, w)
    ref = torch_unet(d, ~P.fluid, P.fluid, sc.dx, w)
    assert np.abs(phi).max() > 0
    assert np.allclose(phi, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())
    # linear in the scale of d
    phi7, _ = PN.unet_phi0(P, 7.0 * d, sc.dx, w)
    assert np.allclose(phi7, 7.0 * phi, rtol=1e-12, atol=1e-15)
