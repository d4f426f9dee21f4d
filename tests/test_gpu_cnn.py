"""GPU parity of the multi-scale CNN initial guess (pyramid, MFMA 3x3
convolutions, 1x1 head, bilinear upsample-sum) and of the hybrid CNN +
Jacobi projection, against the FP64 oracle through the C ABI."""
import numpy as np
import pytest

import scenes
from oracle import grid as G
from oracle import cnn as CN
from oracle import project as PR
from tests.gpu_util import gpu_project, f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def state(nx, ny, seed, nobs):
    sc = scenes.plume_scene(nx, seed=seed, n_obstacles=nobs, ny=ny)
    u, v = scenes.random_faces(nx, ny, seed, kind="mixed")
    return sc, f32(u), f32(v)


@pytest.mark.parametrize("nx,ny,S,C,prec,seed", [
    (64, 64, 3, 16, "fp32", 0),
    (64, 64, 3, 32, "fp32", 1),
    (96, 64, 3, 32, "fp32", 2),     # ragged tiles on the coarse scales
    (256, 256, 3, 32, "fp32", 3),   # the FP32 hybrid network at its size
    (64, 48, 2, 32, "bf16", 4),
    (128, 128, 4, 64, "bf16", 5),
    (80, 40, 1, 16, "fp32", 6),     # single scale, ragged
    (64, 64, 2, 64, "fp32", 8),     # FP32 64 channels: 16 output channels per pass
    (96, 64, 4, 64, "fp32", 9),
])
def test_cnn_prediction_parity(nx, ny, S, C, prec, seed):
    say("cnn", nx, ny, S, C, prec)
    sc, u, v = state(nx, ny, seed, 2)
    w = scenes.random_weights(S, C, seed)
    dt = 0.01
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", dt=dt, params=w, scales=S,
                    channels=C, precision=prec)
    bf = prec == "bf16"
    o = PR.project(sc.flags, u, v, sc.dx, dt=dt, method="cnn", params=w, S=S, C=C, bf16=bf)
    err = rel_l2(g["p"], o["p"], o["plan"].fluid)
    say("  rel L2 vs oracle", err, "s", g["res"].s, o["s"])
    assert g["res"].iters == 0 and g["res"].status == 0
    assert g["res"].s == pytest.approx(o["s"], rel=1e-6)
    assert err <= (1e-3 if bf else 1e-5)
    if bf:
        # distance to the unemulated FP64 network, reported
        o64 = PR.project(sc.flags, u, v, sc.dx, dt=dt, method="cnn", params=w, S=S, C=C)
        say("  bf16 vs fp64 network", rel_l2(g["p"], o64["p"], o["plan"].fluid))
    assert np.all(g["p"][~o["plan"].fluid] == 0)
    assert g["res"].e1_cnn == pytest.approx(o["e1_cnn"], rel=(2e-3 if bf else 1e-5))


def test_cnn_full_size_bf16_512():
    # the 4-scale 64-channel BF16 network on the 512^2 grid, full comparison
    say("cnn 512 bf16")
    sc, u, v = state(512, 512, 7, 3)
    w = scenes.random_weights(4, 64, 7)
    g = gpu_project(sc.flags, u, v, sc.dx, thr=0.0, method="cnn", params=w, scales=4, channels=64,
                    precision="bf16")
    o = PR.project(sc.flags, u, v, sc.dx, method="cnn", params=w, S=4, C=64, bf16=True)
    err = rel_l2(g["p"], o["p"], o["plan"].fluid)
    say("  rel L2", err)
    assert err <= 1e-3


def test_zero_weights_hybrid_is_jacobi_bitwise():
    sc, u, v = state(128, 128, 8, 1)
    z = scenes.zero_weights(3, 32)
    P = G.plan(sc.flags)
    thr = 0.2 * G.e1(P, G.divergence(P, *G.enforce_bc(P, u, v), sc.dx))
    h = gpu_project(sc.flags, u, v, sc.dx, thr=thr, method="hybrid", params=z, scales=3,
                    channels=32)
    j = gpu_project(sc.flags, u, v, sc.dx, thr=thr, method="jacobi")
    assert h["res"].iters == j["res"].iters
    assert np.array_equal(h["p"], j["p"]) and np.array_equal(h["u"], j["u"])


# the last cases are the benchmark's configuration: 512^2, 4 scales of 64
# channels in BF16, E_1 tested every 128 or (the benchmark's) 768 sweeps
# (tagged halo exchanges between the tests, two work-groups per CU)
@pytest.mark.parametrize("n,S,C,prec,seed,thr_rel,ce", [
    (128, 3, 32, "fp32", 0, 0.05, 4), (256, 3, 32, "fp32", 1, 0.1, 4), (128, 4, 64, "bf16", 2, 0.05, 4),
    (512, 4, 64, "bf16", 3, 0.2, 128), (512, 4, 64, "bf16", 4, 0.2, 768)])
def test_hybrid_parity(n, S, C, prec, seed, thr_rel, ce):
    say("hybrid", n, S, C, prec, ce)
    sc, u, v = state(n, n, seed, 2)
    # a small output scale keeps the random net's guess close to zero so
    # that Jacobi from it converges in a moderate number of sweeps
    w = scenes.random_weights(S, C, seed, out_scale=0.05)
    P = G.plan(sc.flags)
    thr = thr_rel * G.e1(P, G.divergence(P, *G.enforce_bc(P, u, v), sc.dx))
    bf = prec == "bf16"
    g = gpu_project(sc.flags, u, v, sc.dx, thr=thr, method="hybrid", params=w, scales=S,
                    channels=C, precision=prec, check_every=ce, max_iters=50000)
    o = PR.project(sc.flags, u, v, sc.dx, threshold=thr, method="hybrid", params=w, S=S, C=C,
                   bf16=bf, check_every=ce, max_iters=50000)
    kg, ko = g["res"].iters, o["iters"]
    say("  iters gpu", kg, "oracle", ko)
    assert g["res"].status == 0 and o["status"] == 0
    assert abs(kg - ko) <= max(ce, 0.01 * ko)
    assert kg % ce == 0
    of = PR.project(sc.flags, u, v, sc.dx, method="hybrid", params=w, S=S, C=C, bf16=bf,
                    fixed_iters=kg) if kg > 0 else o
    err = rel_l2(g["p"], of["p"], P.fluid)
    say("  rel L2 at gpu iters", err)
    assert err <= (1e-3 if bf else 1e-4)
    assert g["res"].e1_final <= 1.01 * thr
