"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/hyproj.h declares, the ctypes structs match the C layouts, and the
host-side argument checks reject bad calls before touching the GPU."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2109_09363_amd as hp
from paper_2109_09363_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hyproj.h")


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z0-9_]+\*?\s+\*?(hyp_[a-z_]+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = hp.lib()
    names = declared_functions()
    assert "hyp_project" in names and "hyp_plan" in names
    for n in names:
        assert hasattr(lib, n), n
        assert n in L.SIGNATURES, f"binding lacks {n}"


def test_struct_layouts_match_c(tmp_path):
    src = tmp_path / "s.c"
    src.write_text('#define __HIP_PLATFORM_AMD__\n#include <stdio.h>\n#include "hyproj.h"\n'
                   'int main(){printf("%zu %zu %zu %zu %zu\\n",sizeof(hyp_result),sizeof(hyp_grid),'
                   'sizeof(hyp_opts),sizeof(hyp_fields),sizeof(hyp_net_desc));return 0;}\n')
    exe = tmp_path / "s"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include",
                           str(src), "-o", str(exe)])
    sizes = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert sizes == [ctypes.sizeof(L.Result), ctypes.sizeof(L.Grid), ctypes.sizeof(L.Opts),
                     ctypes.sizeof(L.Fields), ctypes.sizeof(L.NetDesc)]


def test_host_side_rejections():
    lib = hp.lib()
    assert lib.hyp_version() == 10000
    ctx = ctypes.c_void_p()
    bad = L.NetDesc(3, 48, 0, 0)
    assert lib.hyp_create(ctypes.byref(ctx), ctypes.byref(bad)) == -1
    bad = L.NetDesc(0, 32, 0, 0)
    assert lib.hyp_create(ctypes.byref(ctx), ctypes.byref(bad)) == -1
    # the cascaded networks: fixed widths, known parameter totals, training in FP32 only
    for arch, C, n in ((1, 64, 419459), (2, 32, 126819)):
        c2 = ctypes.c_void_p()
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(0, 0, 1, 0, arch))) == 0
        assert lib.hyp_param_count(c2) == n
        lib.hyp_destroy(c2)
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(3, C, 0, 0, arch))) == 0
        lib.hyp_destroy(c2)
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(3, C + 32, 0, 0, arch))) == -1
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(4, C, 0, 0, arch))) == -1
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(3, C, 0, 1, arch))) == 0
        lib.hyp_destroy(c2)
        assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(3, C, 1, 1, arch))) == -2
    c2 = ctypes.c_void_p()
    assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(0, 0, 1, 0, 3))) == 0
    assert lib.hyp_param_count(c2) == 443441  # the Unet
    lib.hyp_destroy(c2)
    assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(3, 64, 0, 0, 3))) == -1
    # the Unet trains in FP32 (a training context with BF16 storage is refused)
    assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(5, 64, 0, 1, 3))) == 0
    lib.hyp_destroy(c2)
    assert lib.hyp_create(ctypes.byref(c2), ctypes.byref(L.NetDesc(5, 64, 1, 1, 3))) == -2
    assert lib.hyp_create(ctypes.byref(ctx), ctypes.byref(L.NetDesc(3, 32, 0, 0, 4))) == -1
    good = L.NetDesc(3, 32, 0, 0)
    assert lib.hyp_create(ctypes.byref(ctx), ctypes.byref(good)) == 0
    assert lib.hyp_param_count(ctx) == 85155
    nbytes = ctypes.c_size_t()
    g = L.Grid(64, 64, 1 / 64, 0.01, 1.0)
    assert lib.hyp_workspace_size(ctx, ctypes.byref(g), ctypes.byref(nbytes)) == 0
    assert nbytes.value > 64 * 64 * 20
    gbad = L.Grid(1, 64, 1 / 64, 0.01, 1.0)
    assert lib.hyp_workspace_size(ctx, ctypes.byref(gbad), ctypes.byref(nbytes)) == -1
    gbad = L.Grid(64, 64, -1.0, 0.01, 1.0)
    assert lib.hyp_workspace_size(ctx, ctypes.byref(gbad), ctypes.byref(nbytes)) == -1
    # a projection with a too-small workspace is rejected before any launch
    dummy = ctypes.c_void_p(0x1000)
    f = L.Fields(dummy, dummy, None, dummy, dummy, None, None)
    o = L.Opts(1, 100, 1, 0, 1.0, 0, 0, 0, 0, 0)
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           16, None, dummy) == -3
    # hybrid without weights
    o.method = 0
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -6
    # bad options
    o.method = 1
    o.check_every = 0
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.check_every = 1
    o.criterion = 2  # neither E_1 nor E_inf
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.criterion = 0
    o.check_every = 1
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), -1.0, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    for om in (0.0, -1.0, float("nan")):  # the Jacobi weight must be positive
        o.omega = om
        assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                               nbytes.value, None, dummy) == -1
    o.omega = 1.0
    # checkpoints: need fixed_iters, a buffer, a Jacobi method, at most 64 planes
    o.checkpoint_every = 5
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.fixed_iters = 20
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    f.phi_ckpt = dummy
    o.fixed_iters = 5 * 65
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.method = 2
    o.fixed_iters = 20
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.method, o.checkpoint_every, o.fixed_iters, f.phi_ckpt = 1, 0, 0, None
    o.checkpoint_every = -1
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    # tile rows: one of the instantiated heights, Jacobi/hybrid only
    o.checkpoint_every = 0
    o.tile_rows = -4
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.tile_rows = 5
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -2
    o.method, o.tile_rows = 2, 8
    assert lib.hyp_project(ctx, ctypes.byref(g), ctypes.byref(f), 1e-3, ctypes.byref(o), dummy,
                           nbytes.value, None, dummy) == -1
    o.method, o.tile_rows = 1, 0
    assert lib.hyp_set_weights(ctx, dummy, 5) == -1
    assert lib.hyp_destroy(ctx) == 0
    assert lib.hyp_status_str(-4) == b"HIP error"


def test_unbuilt_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(L, "_LIB", None)
    monkeypatch.setattr(L, "LIB_PATH", "/nonexistent/libhyproj.so")
    with pytest.raises(RuntimeError, match="not found"):
        L.lib()
