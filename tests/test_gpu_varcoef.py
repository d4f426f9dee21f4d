"""GPU parity of the variable-density projection (face coefficients
rho0 / rho_face in Eq. 3 and Eq. 2) against the FP64 oracle through the C
ABI: Jacobi at a fixed sweep count and to a threshold, PCG against the exact
solve, the hybrid from the network's guess, the time step with the advected
density, and the reduction to the constant-coefficient path."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from oracle import advect as AD
from oracle import cnn as CN
from oracle import grid as G
from oracle import varcoef as VC
from tests.gpu_util import to_dev, f32, rel_l2

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def case(nx, ny, seed, nobs, drho=0.5):
    """A plume scene with a density field spanning the batched form's ratios."""
    sc = scenes.plume_scene(nx, seed=seed, n_obstacles=nobs, ny=ny)
    u, v = scenes.random_faces(nx, ny, seed, kind="mixed")
    rho = scenes.random_density(nx, ny, seed, sc.rho0, drho)
    return sc, f32(u), f32(v), f32(rho)


def run(sc, u, v, rho, thr, method, params=None, S=0, C=0, dt=1.0, var=True, **opts):
    ny, nx = sc.flags.shape
    pr = hp.Projector(nx, ny, sc.dx, dt, sc.rho0, S, C, "fp32")
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    if params is not None:
        tw = to_dev(params)
        pr.set_weights(tw)
    tu, tv, tr = to_dev(u), to_dev(v), to_dev(rho)
    p = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    pr.project_async(tu, tv, tf, p, thr, method=method, rho=tr, variable_density=var, **opts)
    torch.cuda.synchronize()
    return dict(p=p.cpu().numpy().astype(np.float64), u=tu.cpu().numpy().astype(np.float64),
                v=tv.cpu().numpy().astype(np.float64), res=pr.result())


def oracle(sc, u, v, rho):
    P = G.plan(sc.flags)
    ub, vb = G.enforce_bc(P, u, v)
    d = G.divergence(P, ub, vb, sc.dx)
    bu, bv = VC.face_coefficients(P, rho, sc.rho0)
    return P, ub, vb, d, bu, bv


@pytest.mark.parametrize("nx,ny,seed,nobs,k", [(64, 64, 0, 2, 200), (96, 40, 1, 1, 137),
                                               (200, 136, 2, 3, 400)])
def test_jacobi_fixed_sweeps_match_oracle(nx, ny, seed, nobs, k):
    say("var jacobi fixed", nx, ny, k)
    sc, u, v, rho = case(nx, ny, seed, nobs)
    g = run(sc, u, v, rho, 0.0, "jacobi", fixed_iters=k)
    P, ub, vb, d, bu, bv = oracle(sc, u, v, rho)
    phi = VC.jacobi(P, d, bu, bv, sc.dx, fixed_iters=k)[0]
    uo, vo = VC.correct(P, ub, vb, phi, bu, bv, sc.dx)
    err = rel_l2(g["p"], phi, P.fluid)
    say("  rel L2 phi", err, "u", rel_l2(g["u"], uo), "v", rel_l2(g["v"], vo))
    assert g["res"].iters == k and g["res"].status == 0
    assert err <= 1e-4
    assert rel_l2(g["u"], uo) <= 1e-5 and rel_l2(g["v"], vo) <= 1e-5
    # the returned faces' divergence is the residual of the returned phi
    r = VC.residual(P, d, phi, bu, bv, sc.dx)
    assert g["res"].e1_final == pytest.approx(G.e1(P, r), rel=1e-3)


# intervals above 8 sweeps: the steps between tests synchronise with the
# adjacent tiles only
@pytest.mark.parametrize("n,seed,rel,ce", [(64, 3, 0.05, 4), (128, 4, 0.2, 4), (128, 11, 0.1, 64),
                                           (160, 12, 0.2, 128)])
def test_jacobi_threshold_iterations(n, seed, rel, ce):
    say("var jacobi threshold", n, ce)
    sc, u, v, rho = case(n, n, seed, 2)
    P, ub, vb, d, bu, bv = oracle(sc, u, v, rho)
    thr = rel * G.e1(P, d)
    g = run(sc, u, v, rho, thr, "jacobi", check_every=ce, max_iters=200000)
    phi, ko, st = VC.jacobi(P, d, bu, bv, sc.dx, thr=thr, check_every=ce)
    kg = g["res"].iters
    say("  iters gpu", kg, "oracle", ko)
    assert g["res"].status == 0 and st == VC.STATUS_OK
    assert abs(kg - ko) <= max(ce, 0.01 * ko)
    assert kg % ce == 0
    assert g["res"].e1_final < 1.01 * thr
    # same-algorithm parity at the GPU's sweep count
    phi_k = VC.jacobi(P, d, bu, bv, sc.dx, fixed_iters=kg)[0]
    assert rel_l2(g["p"], phi_k, P.fluid) <= 1e-4


@pytest.mark.parametrize("n,seed", [(48, 5), (64, 6)])
def test_pcg_reaches_exact_solve(n, seed):
    say("var pcg", n)
    sc, u, v, rho = case(n, n, seed, 2)
    P, ub, vb, d, bu, bv = oracle(sc, u, v, rho)
    thr = 1e-5 * G.e1(P, d)
    g = run(sc, u, v, rho, thr, "pcg", max_iters=20000)
    ex = VC.exact_solve(P, d, bu, bv, sc.dx)
    _, ko, _ = VC.pcg(P, d, bu, bv, sc.dx, thr=thr)
    err = rel_l2(g["p"], ex, P.fluid)
    say("  iters gpu", g["res"].iters, "oracle", ko, "rel L2 vs exact", err, "e1", g["res"].e1_final)
    assert g["res"].status == 0
    assert err <= 1e-3
    assert g["res"].e1_final < 1.05 * thr
    assert abs(g["res"].iters - ko) <= max(5, 0.1 * ko)


def test_hybrid_from_the_network_guess():
    n, S, C = 128, 3, 32
    sc, u, v, rho = case(n, n, 7, 2)
    w = scenes.random_weights(S, C, 7, out_scale=0.05)
    P, ub, vb, d, bu, bv = oracle(sc, u, v, rho)
    phi0, s, _ = CN.cnn_phi0(P, d, sc.dx, w, S, C)
    thr = 0.05 * G.e1(P, d)
    g = run(sc, u, v, rho, thr, "hybrid", params=w, S=S, C=C, check_every=4, max_iters=200000)
    phi, ko, st = VC.jacobi(P, d, bu, bv, sc.dx, phi0=phi0, thr=thr, check_every=4)
    kg = g["res"].iters
    say("var hybrid iters gpu", kg, "oracle", ko)
    assert g["res"].status == 0 and abs(kg - ko) <= max(4, 0.01 * ko)
    phi_k = VC.jacobi(P, d, bu, bv, sc.dx, phi0=phi0, fixed_iters=kg)[0]
    assert rel_l2(g["p"], phi_k, P.fluid) <= 1e-4


def test_uniform_density_equals_constant_path():
    # rho = rho0 everywhere: every beta is 1 and the variable-density kernels
    # compute the constant-coefficient projection
    sc, u, v, _ = case(96, 96, 8, 2)
    rho = np.full(sc.flags.shape, sc.rho0)
    for method, kw in (("jacobi", dict(fixed_iters=300)), ("pcg", dict(max_iters=5000))):
        thr = 0.0 if method == "jacobi" else 1e-2
        a = run(sc, u, v, rho, thr, method, var=True, **kw)
        b = run(sc, u, v, rho, thr, method, var=False, **kw)
        say("uniform", method, a["res"].iters, b["res"].iters, rel_l2(a["p"], b["p"]))
        assert a["res"].iters == b["res"].iters
        assert rel_l2(a["p"], b["p"]) <= 1e-6 and rel_l2(a["u"], b["u"]) <= 1e-6


def test_step_with_advected_density():
    # one time step from a seeded state: advection moves the density, and the
    # projection uses the advected density in its operator
    n = 64
    sc, u, v, rho = case(n, n, 9, 1, drho=0.4)
    u, v = f32(0.5 * u), f32(0.5 * v)
    xi = f32(scenes.inflow_noise(9, 0, n))
    pr = hp.Projector(n, n, sc.dx, 1.0, sc.rho0)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    tr, tu, tv = to_dev(rho), to_dev(u), to_dev(v)
    p = torch.zeros((n, n), dtype=torch.float32, device="cuda")
    pr.step_async(tr, tu, tv, tf, p, to_dev(xi), threshold=0.0, g=sc.g, drho=0.4, u_in=sc.u_in,
                  method="jacobi", fixed_iters=60, variable_density=True)
    torch.cuda.synchronize()
    res = pr.result()
    P = G.plan(sc.flags)
    dt = AD.cfl_dt(u, v, sc.dx, sc.u_in)
    assert res.dt == pytest.approx(dt, rel=1e-6)
    ro, us, vs = AD.advect_step(P, sc.flags, rho, u, v, sc.dx, dt, sc.g, sc.rho0, 0.4, sc.u_in, xi)
    # the oracle's own advected density enters its operator
    bu, bv = VC.face_coefficients(P, ro, sc.rho0)
    d = G.divergence(P, us, vs, sc.dx)
    phi = VC.jacobi(P, d, bu, bv, sc.dx, fixed_iters=60)[0]
    uo, vo = VC.correct(P, us, vs, phi, bu, bv, sc.dx)
    eu, ev = rel_l2(tu.cpu().numpy(), uo), rel_l2(tv.cpu().numpy(), vo)
    say("var step rel L2 u", eu, "v", ev)
    assert eu <= 1e-4 and ev <= 1e-4


def test_rejections():
    from paper_2109_09363_amd import _lib as L
    n = 32
    sc, u, v, rho = case(n, n, 10, 0)
    pr = hp.Projector(n, n, sc.dx)
    tf = to_dev(sc.flags, torch.uint8)
    pr.plan(tf)
    p = torch.empty((n, n), dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        pr.project_async(to_dev(u), to_dev(v), tf, p, 1e-3, method="jacobi", variable_density=True)
