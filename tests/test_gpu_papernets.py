"""GPU parity of the paper's cascaded MultiScale and SmallScale networks
(Sec. 3.1, Fig. 3: branches at n/4, n/2, n; 5x5, 3x3 and 1x1 convolutions on
MFMA; coarse output upsampled and concatenated), of its Unet (Fig. 4: max
pooling, bilinear upsampling, skip concatenation) and of the hybrid
projection that starts from their guess, against the FP64 oracle through the
C ABI."""
import numpy as np
import pytest

import scenes
import paper_2109_09363_amd as hp
from oracle import grid as G
from oracle import papernets as PN
from oracle import solve as SV
from tests.gpu_util import gpu_project, f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def state(nx, ny, seed, nobs):
    sc = scenes.plume_scene(nx, seed=seed, n_obstacles=nobs, ny=ny)
    u, v = scenes.random_faces(nx, ny, seed, kind="mixed")
    return sc, f32(u), f32(v)


# BF16 bar of the cascade.  The oracle emulates every BF16 storage point, but
# each finer branch re-quantizes the upsampled output of the coarser one,
# which already differs from the oracle's by the BF16 rounding decisions that
# FP32 and FP64 accumulation took differently; the rate of flipped roundings
# grows with that upstream difference (measured: 3e-5 for the parallel net,
# 1e-4 for one branch alone, 3e-3 .. 4e-3 for the cascade).  So the cascade is
# held to 1e-2 (2.5 BF16 ulps, 2^-8 = 3.9e-3) against the emulation and to
# 3e-2 against the unemulated FP64 network; the Unet, 19 layers deep with the
# encoder's output re-quantized after pooling and upsampling, to the same.
BF16_EMULATED, BF16_FP64 = 1e-2, 3e-2


def oracle_phi0(sc, u, v, w, arch, bf16):
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    phi0, s, _ = PN.phi0(P, d, sc.dx, w, arch, bf16=bf16)
    return P, d, phi0, s


def test_param_counts_match_the_oracle():
    for arch in PN.ARCHS + ("unet",):
        pr = hp.Projector(32, 32, 1 / 32, arch=arch)
        assert pr.param_count == PN.param_count(arch) == scenes.random_paper_weights(arch, 0).size


@pytest.mark.parametrize("arch,nx,ny,prec,seed", [
    ("multiscale", 64, 64, "fp32", 0),
    ("smallscale", 64, 64, "fp32", 1),
    ("multiscale", 96, 40, "fp32", 2),    # ragged tiles on every branch
    ("smallscale", 48, 80, "bf16", 3),
    ("multiscale", 128, 128, "bf16", 4),
    ("multiscale", 256, 256, "fp32", 5),  # several tiles per CU on the finest branch
    ("smallscale", 20, 12, "fp32", 6),    # coarsest branch 5x3: one partial tile
])
def test_papernet_prediction_parity(arch, nx, ny, prec, seed):
    say("papernet", arch, nx, ny, prec)
    sc, u, v = state(nx, ny, seed, 2)
    w = scenes.random_paper_weights(arch, seed)
    dt, rho0 = 0.01, 1.0
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", dt=dt, rho0=rho0, params=w,
                    precision=prec, arch=arch)
    bf = prec == "bf16"
    P, d, phi0, s = oracle_phi0(sc, u, v, w, arch, bf)
    p_or = rho0 * phi0 / dt
    err = rel_l2(g["p"], p_or, P.fluid)
    say("  rel L2 vs oracle", err, "s", g["res"].s, s)
    assert g["res"].iters == 0 and g["res"].status == 0
    assert g["res"].s == pytest.approx(s, rel=1e-6)
    assert err <= (BF16_EMULATED if bf else 1e-5)
    assert np.all(g["p"][~P.fluid] == 0)
    e1_cnn = G.e1(P, G.residual(P, d, phi0, sc.dx))
    assert g["res"].e1_cnn == pytest.approx(e1_cnn, rel=(BF16_EMULATED if bf else 1e-5))
    if bf:
        _, _, phi64, _ = oracle_phi0(sc, u, v, w, arch, False)
        e64 = rel_l2(g["p"], rho0 * phi64 / dt, P.fluid)
        say("  bf16 vs fp64 network", e64)
        assert e64 <= BF16_FP64


def test_papernet_full_size_512_bf16():
    say("papernet multiscale 512 bf16")
    sc, u, v = state(512, 512, 7, 3)
    w = scenes.random_paper_weights("multiscale", 7)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", params=w, precision="bf16",
                    arch="multiscale")
    P, d, phi0, s = oracle_phi0(sc, u, v, w, "multiscale", True)
    err = rel_l2(g["p"], phi0, P.fluid)
    say("  rel L2", err)
    assert err <= BF16_EMULATED


@pytest.mark.parametrize("arch,n,prec,seed,thr_rel", [("multiscale", 128, "fp32", 0, 0.05),
                                                      ("smallscale", 96, "bf16", 1, 0.1)])
def test_papernet_hybrid_parity(arch, n, prec, seed, thr_rel):
    say("papernet hybrid", arch, n, prec)
    sc, u, v = state(n, n, seed, 2)
    w = scenes.random_paper_weights(arch, seed, out_scale=0.05)
    bf = prec == "bf16"
    P, d, phi0, s = oracle_phi0(sc, u, v, w, arch, bf)
    thr = thr_rel * G.e1(P, d)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=thr, method="hybrid", params=w, precision=prec,
                    arch=arch, check_every=4, max_iters=50000)
    phi_o, ko, st, _ = SV.jacobi(P, d, sc.dx, phi0, thr, 1.0, 4, 50000)
    kg = g["res"].iters
    say("  iters gpu", kg, "oracle", ko)
    assert g["res"].status == 0 and st == SV.STATUS_OK
    assert abs(kg - ko) <= max(4, 0.01 * ko)
    phi_f = SV.jacobi(P, d, sc.dx, phi0, 0.0, 1.0, 1, kg, kg)[0] if kg > 0 else phi0
    err = rel_l2(g["p"], phi_f, P.fluid)
    say("  rel L2 at gpu iters", err)
    assert err <= (BF16_EMULATED if bf else 1e-4)
    assert g["res"].e1_final <= 1.01 * thr


def unet_oracle(sc, u, v, w, bf16):
    P = G.plan(sc.flags)
    d = G.divergence(P, *G.enforce_bc(P, u, v), sc.dx)
    phi0, s = PN.unet_phi0(P, d, sc.dx, w, bf16=bf16)
    return P, d, phi0, s


@pytest.mark.parametrize("nx,ny,prec,seed", [
    (64, 64, "fp32", 0),
    (96, 48, "fp32", 1),     # ragged tiles at every scale, 6x3 at the bottom
    (64, 64, "bf16", 2),
    (112, 80, "bf16", 3),
    (256, 256, "fp32", 4),   # the 128-channel decoder inputs in two chunks (FP32)
])
def test_unet_prediction_parity(nx, ny, prec, seed):
    say("unet", nx, ny, prec)
    sc, u, v = state(nx, ny, seed, 2)
    w = scenes.random_paper_weights("unet", seed)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", params=w, precision=prec,
                    arch="unet")
    bf = prec == "bf16"
    P, d, phi0, s = unet_oracle(sc, u, v, w, bf)
    err = rel_l2(g["p"], phi0, P.fluid)
    say("  rel L2 vs oracle", err)
    assert g["res"].status == 0 and g["res"].s == pytest.approx(s, rel=1e-6)
    assert err <= (BF16_EMULATED if bf else 1e-5)
    assert np.all(g["p"][~P.fluid] == 0)
    if bf:
        e64 = rel_l2(g["p"], unet_oracle(sc, u, v, w, False)[2], P.fluid)
        say("  bf16 vs fp64 network", e64)
        assert e64 <= BF16_FP64


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_unet_full_size_512(prec):
    say("unet 512", prec)
    sc, u, v = state(512, 512, 8, 3)
    w = scenes.random_paper_weights("unet", 8)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", params=w, precision=prec,
                    arch="unet")
    P, d, phi0, s = unet_oracle(sc, u, v, w, prec == "bf16")
    err = rel_l2(g["p"], phi0, P.fluid)
    say("  rel L2", err)
    assert err <= (BF16_EMULATED if prec == "bf16" else 1e-5)


def test_unet_hybrid_parity():
    n = 128
    say("unet hybrid", n)
    sc, u, v = state(n, n, 5, 2)
    w = scenes.random_paper_weights("unet", 5, out_scale=0.05)
    P, d, phi0, s = unet_oracle(sc, u, v, w, False)
    thr = 0.05 * G.e1(P, d)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=thr, method="hybrid", params=w, arch="unet",
                    check_every=4, max_iters=50000)
    phi_o, ko, st, _ = SV.jacobi(P, d, sc.dx, phi0, thr, 1.0, 4, 50000)
    kg = g["res"].iters
    say("  iters gpu", kg, "oracle", ko)
    assert g["res"].status == 0 and st == SV.STATUS_OK
    assert abs(kg - ko) <= max(4, 0.01 * ko)
    phi_f = SV.jacobi(P, d, sc.dx, phi0, 0.0, 1.0, 1, kg, kg)[0] if kg > 0 else phi0
    assert rel_l2(g["p"], phi_f, P.fluid) <= 1e-4


def test_papernet_rejects_training_and_bad_shapes():
    from paper_2109_09363_amd import _lib as L
    with pytest.raises(L.HypError):  # the paper's networks train in FP32 only
        hp.Projector(64, 64, 1 / 64, precision="bf16", arch="multiscale", train=True)
    with pytest.raises(L.HypError):
        hp.Projector(64, 64, 1 / 64, channels=32, arch="multiscale")
    with pytest.raises(L.HypError):  # the Unet trains in FP32 only
        hp.Projector(64, 64, 1 / 64, precision="bf16", arch="unet", train=True)
    pr = hp.Projector(62, 64, 1 / 64, arch="smallscale")  # sides must be multiples of 4
    import torch
    t = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    w = torch.from_numpy(scenes.random_paper_weights("smallscale", 0)).cuda()
    pr.set_weights(w)
    flags = torch.zeros((64, 62), dtype=torch.uint8, device="cuda")
    pr.plan(flags)
    with pytest.raises(L.HypError):
        pr.project_async(t(64, 63), t(65, 62), flags, t(64, 62), 1e-3, method="cnn")
