"""Errors of the experiments' results against the FP64 oracle.

python -m tests.experiment_errors DIR [--replica-max-iters N] [--out FILE]

DIR is what `python -m paper_2109_09363_amd.experiments WHAT --save ROOT`
wrote under ROOT/WHAT: per plume (or per sampled batch instance) the first
timed step's projection inputs (flags, advected faces, dx, dt, rho0) and, per
method, the pressure the GPU returned with its sweep or iteration count.  For
each case this prints one JSON line with

  p_vs_exact       relative L2 (fluid cells) of the GPU's pressure against
                   the exact FP64 solve of Eq. (3) (what a threshold stop
                   leaves of the pressure: the method's error, not the GPU's)
  uv_vs_exact      relative L2 over all faces of the velocity that pressure
                   leaves (u* - grad phi, phi = dt p / rho0, the correction of
                   Eq. 2 applied by the oracle) against the exactly projected
                   velocity: what the next time step carries forward
  p_vs_replica     relative L2 against the oracle running the same algorithm
                   on the same faces: the hybrid with the same network
                   (BF16 rounding emulated where the GPU used BF16) and the
                   GPU's sweep count, or PCG to the same threshold with its
                   test every iteration (its iteration count beside it);
                   skipped above --replica-max-iters sweeps (plain FP64
                   numpy Jacobi costs about 2 ms per sweep at 512^2)

and a final line with the means per (method, precision, weights,
threshold).  This is test-side code: the library never runs the oracle.
"""
from __future__ import annotations

import argparse
import glob
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import scenes  # noqa: E402
from oracle import grid as G, project as PR, solve as SV, varcoef as VC  # noqa: E402
from oracle.cnn import cnn_phi0  # noqa: E402

WEIGHTS = os.path.join(ROOT, "paper_2109_09363_amd", "weights", "plume_s4c64.npy")
S4, C64 = 4, 64


def network(name):
    if name == "trained":
        return np.load(WEIGHTS, allow_pickle=False).astype(np.float32).astype(np.float64)
    if name == "zero":
        return np.zeros(scenes.cnn_param_count(S4, C64))
    if name == "random":
        return scenes.random_weights(S4, C64, 7).astype(np.float32).astype(np.float64)
    return None


def rel(P, a, b):
    return float(np.linalg.norm((a - b)[P.fluid]) / max(np.linalg.norm(b[P.fluid]), 1e-300))


def evaluate(path, replica_max):
    base = path[:-4]
    z = np.load(path, allow_pickle=False)
    with open(base + ".json") as f:
        meta = json.load(f)
    flags = z["flags"]
    u, v = z["u"].astype(np.float64), z["v"].astype(np.float64)
    dx, dt, rho0 = (float(x) for x in z["scalars"])
    P = G.plan(flags)
    ub, vb = G.enforce_bc(P, u, v)
    d = G.divergence(P, ub, vb, dx)
    rho = None
    if os.path.exists(base + "_rho.npy"):
        rho = np.load(base + "_rho.npy", allow_pickle=False).astype(np.float64)
    exact = None
    out = []
    for i, c in enumerate(meta):
        p = z[f"p{i}"].astype(np.float64)
        row = dict(case=os.path.basename(base), **c)
        var = bool(c.get("variable_density", False))
        if var:
            bu, bv = VC.face_coefficients(P, rho, rho0)
        elif exact is None:
            exact = rho0 / dt * SV.exact_solve(P, d, dx)
        if not var:
            row["p_vs_exact"] = rel(P, p, exact)
            ue, ve = G.correct(P, ub, vb, exact * dt / rho0, dx)
            ug, vg = G.correct(P, ub, vb, p * dt / rho0, dx)
            row["uv_vs_exact"] = float(np.sqrt((np.sum((ug - ue) ** 2) + np.sum((vg - ve) ** 2))
                                               / (np.sum(ue ** 2) + np.sum(ve ** 2))))
        k = int(c["iters"])
        if c["method"] == "pcg" and not var:
            o = PR.project(flags, u, v, dx, dt=dt, rho0=rho0, method="pcg", threshold=c["threshold"],
                           check_every=1)
            row["p_vs_replica"] = rel(P, p, o["p"])
            row["replica_iters"] = int(o["iters"])
        elif k <= replica_max:
            w = network(c.get("weights", "trained"))
            bf16 = c.get("precision") == "bf16"
            if w is not None:
                phi0 = cnn_phi0(P, d, dx, w, S4, C64, bf16=bf16)[0]
            else:
                phi0 = np.zeros(P.shape)
            if var:
                phi = VC.jacobi(P, d, bu, bv, dx, phi0=phi0, fixed_iters=k)[0] if k > 0 else phi0
            else:
                phi = SV.jacobi(P, d, dx, phi0, fixed_iters=k)[0] if k > 0 else phi0
            row["p_vs_replica"] = rel(P, p, rho0 * phi / dt)
            row["replica_iters"] = k
        out.append(row)
        print(json.dumps(row), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--replica-max-iters", type=int, default=20000)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    rows = []
    for path in sorted(glob.glob(os.path.join(a.dir, "*.npz"))):
        rows += evaluate(path, a.replica_max_iters)
    groups = {}
    for r in rows:
        key = f'{r["method"]}/{r.get("precision", "")}/{r.get("weights", "")}/{r["threshold"]:g}'
        groups.setdefault(key, []).append(r)
    summary = {}
    for key, rs in groups.items():
        e = [r["p_vs_exact"] for r in rs if "p_vs_exact" in r]
        q = [r["p_vs_replica"] for r in rs if "p_vs_replica" in r]
        uv = [r["uv_vs_exact"] for r in rs if "uv_vs_exact" in r]
        summary[key] = {"cases": len(rs),
                        "mean_p_vs_exact": float(np.mean(e)) if e else None,
                        "mean_uv_vs_exact": float(np.mean(uv)) if uv else None,
                        "max_p_vs_replica": float(np.max(q)) if q else None,
                        "replicated": len(q)}
    line = json.dumps({"summary": summary})
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            for r in rows:
                f.write(json.dumps(r) + "\n")
            f.write(line + "\n")


if __name__ == "__main__":
    main()
