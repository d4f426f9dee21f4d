"""Pins of the oracle CNN (Sec. 3.1): convolution against a brute-force loop
and PyTorch's CPU conv with replication padding, resampling against closed
forms and PyTorch's bilinear interpolation, parameter counts, invariances."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import cnn as CN
from oracle import grid as G
from oracle import solve as SV
from oracle import project as PR
import scenes


def brute_conv(x, W, b):
    H, Wd, cin = x.shape
    cout = W.shape[0]
    out = np.zeros((H, Wd, cout))
    for y in range(H):
        for xx in range(Wd):
            for co in range(cout):
                acc = b[co]
                for ky in range(3):
                    for kx in range(3):
                        yy = min(max(y + ky - 1, 0), H - 1)
                        xs = min(max(xx + kx - 1, 0), Wd - 1)
                        for ci in range(cin):
                            acc += W[co, ky, kx, ci] * x[yy, xs, ci]
                out[y, xx, co] = acc
    return out


def test_conv_bruteforce_6x6():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((6, 5, 3))
    W = rng.standard_normal((4, 3, 3, 3))
    b = rng.standard_normal(4)
    assert np.allclose(CN.conv3x3_replicate(x, W, b), brute_conv(x, W, b), atol=1e-13)


def test_conv_matches_torch_replicate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((9, 7, 5))
    W = rng.standard_normal((6, 3, 3, 5))
    b = rng.standard_normal(6)
    xt = torch.from_numpy(x).permute(2, 0, 1)[None]
    wt = torch.from_numpy(W).permute(0, 3, 1, 2)
    ref = F.conv2d(F.pad(xt, (1, 1, 1, 1), mode="replicate"), wt, torch.from_numpy(b))
    ref = ref[0].permute(1, 2, 0).numpy()
    assert np.allclose(CN.conv3x3_replicate(x, W, b), ref, atol=1e-12)


def test_down2_is_bilinear_half():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((8, 6, 2))
    ref = F.interpolate(torch.from_numpy(x).permute(2, 0, 1)[None], scale_factor=0.5,
                        mode="bilinear", align_corners=False)[0].permute(1, 2, 0).numpy()
    assert np.allclose(CN.down2(x), ref, atol=1e-14)


def test_up2_weights_and_torch():
    rng = np.random.default_rng(3)
    t = rng.standard_normal((5, 7))
    up = CN.up2(t)
    ref = F.interpolate(torch.from_numpy(t)[None, None], scale_factor=2, mode="bilinear",
                        align_corners=False)[0, 0].numpy()
    assert np.allclose(up, ref, atol=1e-14)
    # interior weights 9/16, 3/16, 3/16, 1/16
    e = np.zeros((5, 7)); e[2, 3] = 1.0
    u = CN.up2(e)
    assert u[4, 6] == 9 / 16 and u[4, 5] == 3 / 16 and u[3, 6] == 3 / 16 and u[3, 5] == 1 / 16
    # edge clamp: a constant field stays constant
    assert np.allclose(CN.up2(np.ones((3, 4))), 1.0)


def test_param_counts():
    assert CN.param_count(3, 32) == 85155
    assert CN.param_count(4, 64) == 448260
    assert scenes.cnn_param_count(3, 32) == 85155


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(5000) * 10 ** rng.uniform(-6, 6, 5000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.0e38, -2.5e-30]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(CN.bf16_round(x), ref)


def _plume_state(n, seed, n_obs=1):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=n_obs)
    u, v = scenes.random_faces(n, n, seed, kind="mixed")
    P = G.plan(sc.flags)
    u, v = G.enforce_bc(P, u, v)
    return sc, P, u, v


def test_scale_invariance():
    sc, P, u, v = _plume_state(16, 0)
    w = scenes.random_weights(3, 4, 0)
    d = G.divergence(P, u, v, sc.dx)
    p1, s1, _ = CN.cnn_phi0(P, d, sc.dx, w, 3, 4)
    p2, s2, _ = CN.cnn_phi0(P, 3.5 * d, sc.dx, w, 3, 4)
    assert s2 == pytest.approx(3.5 * s1, rel=1e-14)
    assert np.allclose(p2, 3.5 * p1, rtol=1e-12, atol=1e-300)
    assert np.all(p1[~P.fluid] == 0)


def test_zero_weights_hybrid_equals_jacobi():
    sc, P, u, v = _plume_state(16, 1)
    z = scenes.zero_weights(3, 8)
    h = PR.project(sc.flags, u, v, sc.dx, method="hybrid", params=z, S=3, C=8,
                   threshold=1e-2, check_every=3)
    j = PR.project(sc.flags, u, v, sc.dx, method="jacobi", threshold=1e-2, check_every=3)
    assert h["iters"] == j["iters"]
    assert np.array_equal(h["phi"], j["phi"]) and np.array_equal(h["u"], j["u"])


def test_exact_guess_takes_zero_sweeps():
    sc, P, u, v = _plume_state(16, 2)
    d = G.divergence(P, u, v, sc.dx)
    ex = SV.exact_solve(P, d, sc.dx)
    r = PR.project(sc.flags, u, v, sc.dx, method="jacobi", threshold=1e-8, phi_init=ex)
    assert r["iters"] == 0 and r["e1_final"] < 1e-8


def test_single_scale_single_channel_closed_form():
    # S = 1, C = 1: t = wo * relu(...) + bo; with identity-like weights the
    # net reduces to a hand-computable map.
    sc, P, u, v = _plume_state(8, 3, n_obs=0)
    d = G.divergence(P, u, v, sc.dx)
    w = np.zeros(CN.param_count(1, 1))
    # layer 0: centre tap of channel 0 = 1 (W[0][1][1][0]); layers 1..3: centre tap = 1
    o = 0
    w[o + 4 * 2 + 0] = 1.0; o += 18 + 1
    for _ in range(3):
        w[o + 4] = 1.0; o += 9 + 1
    w[o] = 2.0; w[o + 1] = 0.0
    phi0, s, _ = CN.cnn_phi0(P, d, sc.dx, w, 1, 1)
    s_ref = np.sqrt(np.mean(d[P.fluid] ** 2))
    ref = np.where(P.fluid, sc.dx ** 2 * s_ref * 2.0 * np.maximum(d / s_ref, 0.0), 0.0)
    assert np.allclose(phi0, ref, atol=1e-15)


# ---- the whole multi-scale network against an independent PyTorch CPU
# rendering (Sec. 3.1: the same input at several resolutions, bilinear
# resampling, replication padding, ReLU on the hidden layers, a linear
# output per scale, outputs summed from the coarsest scale to the finest).

def _bf16(t):
    """Storage rounding of the BF16 path: FP32 value, then round to nearest
    even bfloat16."""
    return t.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def torch_parallel(d, fluid, dx, params, S, C, bf16=False):
    s = float(np.sqrt(np.sum(d[fluid] ** 2) / fluid.sum()))
    x = torch.from_numpy(np.stack([np.where(fluid, d / s, 0.0), (~fluid).astype(np.float64)]))[None]
    levels = [x]
    for _ in range(S - 1):
        levels.append(F.interpolate(levels[-1], scale_factor=0.5, mode="bilinear",
                                    align_corners=False))
    rnd = _bf16 if bf16 else (lambda t: t)
    p = torch.from_numpy(np.asarray(params, np.float64))
    o, ys = 0, []
    for k in range(S):
        h = rnd(levels[k])
        cin = 2
        for _ in range(4):
            W = p[o:o + C * 9 * cin].reshape(C, 3, 3, cin).permute(0, 3, 1, 2); o += C * 9 * cin
            b = p[o:o + C]; o += C
            h = rnd(torch.relu(F.conv2d(F.pad(h, (1, 1, 1, 1), mode="replicate"), rnd(W), b)))
            cin = C
        wo = p[o:o + C].reshape(1, C, 1, 1); o += C
        bo = p[o:o + 1]; o += 1
        ys.append(F.conv2d(h, wo, bo))
    t = ys[S - 1]
    for k in range(S - 2, -1, -1):
        t = ys[k] + F.interpolate(t, scale_factor=2, mode="bilinear", align_corners=False)
    return np.where(fluid, dx * dx * s * t[0, 0].numpy(), 0.0)


@pytest.mark.parametrize("S,C,n,seed,bf16", [(2, 4, 16, 0, False), (3, 8, 24, 1, False),
                                              (4, 4, 32, 2, False), (3, 8, 24, 3, True),
                                              (4, 8, 32, 4, True)])
def test_multiscale_net_matches_torch_rendering(S, C, n, seed, bf16):
    sc, P, u, v = _plume_state(n, seed, n_obs=2)
    w = scenes.random_weights(S, C, seed, out_scale=0.5)
    d = G.divergence(P, u, v, sc.dx)
    phi, s, cache = CN.cnn_phi0(P, d, sc.dx, w, S, C, bf16=bf16, keep=True)
    ref = torch_parallel(d, P.fluid, sc.dx, w, S, C, bf16=bf16)
    assert np.abs(phi).max() > 0
    assert np.allclose(phi, ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    # every scale contributes (the test would not see a dropped scale otherwise)
    for y in cache["ys"]:
        assert np.abs(y).max() > 1e-3 * np.abs(cache["t"]).max()


def _nearest_up2(t):
    return np.repeat(np.repeat(t, 2, axis=0), 2, axis=1)


@pytest.mark.parametrize("mutant", ["nearest_up", "scales_reversed", "no_coarse_sum"])
def test_torch_rendering_detects_a_wrong_combination(mutant, monkeypatch):
    """Plausible mistakes in the coarse-to-fine combination, planted in the
    oracle on the CPU, fail the comparison with the PyTorch rendering."""
    S, C, n, seed = 3, 8, 24, 1
    sc, P, u, v = _plume_state(n, seed, n_obs=2)
    w = scenes.random_weights(S, C, seed, out_scale=0.5)
    d = G.divergence(P, u, v, sc.dx)
    ref = torch_parallel(d, P.fluid, sc.dx, w, S, C)
    if mutant == "nearest_up":
        monkeypatch.setattr(CN, "up2", _nearest_up2)
        phi = CN.cnn_phi0(P, d, sc.dx, w, S, C)[0]
    elif mutant == "scales_reversed":
        per = CN.param_count(1, C)
        wr = np.concatenate([w[k * per:(k + 1) * per] for k in reversed(range(S))])
        phi = CN.cnn_phi0(P, d, sc.dx, wr, S, C)[0]
    else:
        real_up2 = CN.up2
        monkeypatch.setattr(CN, "up2", lambda t: 0.0 * real_up2(t))
        phi = CN.cnn_phi0(P, d, sc.dx, w, S, C)[0]
    assert not np.allclose(phi, ref, rtol=0, atol=1e-3 * np.abs(ref).max())
