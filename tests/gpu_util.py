"""Helpers for the GPU parity tests: run the HIP projection on numpy inputs
(through the C ABI) and compare with the oracle on the same FP32-rounded
inputs."""
import numpy as np
import torch

import paper_2109_09363_amd as hp


def to_dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype).cuda()


def gpu_project(flags, u, v, dx, thr, method="jacobi", dt=1.0, rho0=1.0, params=None,
                scales=0, channels=0, precision="fp32", p_init=None, arch="parallel", **opts):
    ny, nx = flags.shape
    pr = hp.Projector(nx, ny, dx, dt, rho0, scales, channels, precision, arch=arch)
    tf = to_dev(flags, torch.uint8)
    pr.plan(tf)
    if params is not None:
        tp = to_dev(params)
        pr.set_weights(tp)
    tu, tv = to_dev(u), to_dev(v)
    p = torch.empty((ny, nx), dtype=torch.float32, device="cuda")
    tpi = None if p_init is None else to_dev(p_init)
    pr.project_async(tu, tv, tf, p, thr, method=method, p_init=tpi, **opts)
    torch.cuda.synchronize()
    res = pr.result()
    return dict(p=p.cpu().numpy().astype(np.float64), u=tu.cpu().numpy().astype(np.float64),
                v=tv.cpu().numpy().astype(np.float64), res=res)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel_l2(a, b, mask=None):
    if mask is not None:
        a = a[mask]
        b = b[mask]
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)
