"""The no-allocation projection entry point (hyp_project_noalloc): through
the C ABI, its results equal those of hyp_plan + hyp_project on a caller
workspace, on two calls in a row (the second on a smaller grid, in the same
static array), and a grid beyond the array's size is rejected before
anything is enqueued."""
import numpy as np
import pytest
import torch

import scenes
import paper_2109_09363_amd as hp
from paper_2109_09363_amd import _lib as L
from tests.gpu_util import to_dev, f32

pytestmark = pytest.mark.gpu


def _case(n, ny, seed, nobs):
    sc = scenes.plume_scene(n, seed=seed, n_obstacles=nobs, ny=ny)
    u, v = scenes.random_faces(sc.nx, sc.ny, seed, kind="mixed")
    return sc, f32(u), f32(v)


def _run(pr, sc, u, v, noalloc, **opts):
    tf = to_dev(sc.flags, torch.uint8)
    tu, tv = to_dev(u), to_dev(v)
    p = torch.zeros((sc.ny, sc.nx), dtype=torch.float32, device="cuda")
    if noalloc:
        pr.project_noalloc_async(tu, tv, tf, p, **opts)
    else:
        pr.plan(tf)
        pr.project_async(tu, tv, tf, p, **opts)
    torch.cuda.synchronize()
    r = pr.result()
    return p.cpu().numpy(), tu.cpu().numpy(), tv.cpu().numpy(), r


def _same(a, b):
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    ra, rb = a[3], b[3]
    assert (ra.iters, ra.status) == (rb.iters, rb.status)
    assert ra.e1_final == rb.e1_final and ra.e1_init == rb.e1_init


def test_noalloc_matches_workspace_path_twice():
    # first call: 512^2 hybrid with the 4-scale 64-channel BF16 network
    S, C = 4, 64
    sc, u, v = _case(512, None, 21, 3)
    w = to_dev(scenes.random_weights(S, C, 21, out_scale=0.05))
    pr = hp.Projector(512, 512, sc.dx, 0.01, 1.0, S, C, "bf16")
    pr.set_weights(w)
    opts = dict(threshold=1.0, method="hybrid", check_every=16, max_iters=4000)
    ref = _run(pr, sc, u, v, False, **opts)
    got = _run(pr, sc, u, v, True, **opts)
    print("512^2 hybrid: sweeps", got[3].iters, "status", got[3].status, flush=True)
    _same(got, ref)
    # second call: a smaller grid (PCG and Jacobi) in the same array
    sc2, u2, v2 = _case(200, 150, 22, 2)
    pr2 = hp.Projector(200, 150, sc2.dx, 0.01, 1.0)
    for method, o in (("pcg", dict(threshold=1e-3 * 50)), ("jacobi", dict(threshold=0.0, fixed_iters=300))):
        ref = _run(pr2, sc2, u2, v2, False, method=method, **o)
        got = _run(pr2, sc2, u2, v2, True, method=method, **o)
        print("200x150", method, "iters", got[3].iters, flush=True)
        _same(got, ref)


def test_noalloc_rejects_grids_beyond_the_array():
    pr = hp.Projector(2048, 2048, 1 / 2048)
    t = lambda *s: torch.zeros(s, dtype=torch.float32, device="cuda")
    flags = torch.zeros((2048, 2048), dtype=torch.uint8, device="cuda")
    with pytest.raises(L.HypError) as e:
        pr.project_noalloc_async(t(2048, 2049), t(2049, 2048), flags, t(2048, 2048), 1e-3,
                                 method="jacobi")
    assert e.value.code == -3  # HYP_EWORKSPACE
