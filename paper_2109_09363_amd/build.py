"""Build the hyproj HIP library (gfx950) in-tree: paper_2109_09363_amd/libhyproj.so.

Each source is compiled to an object of its own (in parallel), then the
objects are linked into the shared library; every translation unit launches
only its own kernels, so no relocatable device code is needed."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
OUT = os.path.join(HERE, "libhyproj.so")
SOURCES = ["api.hip", "stencil.hip", "solvers.hip", "cnn.hip", "advect.hip", "backward.hip", "batched.hip",
           "papernets.hip", "noalloc.hip"]
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    noise = [l for l in (r.stdout + r.stderr).splitlines()
             if l.strip() and "packed-fp32-ops" not in l]
    return r.returncode, "\n".join(noise)


def build(verbose: bool = False, jobs: int | None = None) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    objs, cmds = [], []
    for s in SOURCES:
        o = os.path.join(OBJ, s.replace(".hip", ".o"))
        objs.append(o)
        cmds.append([hipcc, *FLAGS, *inc, "-c", "-o", o, os.path.join(SRC, s)])
    jobs = jobs or min(len(cmds), max(1, min(16, os.cpu_count() or 1)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(lambda c: _run(c, verbose), cmds))
    failed = False
    for (rc, msg), c in zip(results, cmds):
        if msg and (rc != 0 or verbose):
            sys.stderr.write(msg + "\n")
        failed = failed or rc != 0
    if failed:
        raise RuntimeError("hipcc failed")
    tmp = OUT + ".tmp"
    rc, msg = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
    if rc != 0:
        sys.stderr.write(msg + "\n")
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
