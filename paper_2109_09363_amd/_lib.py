"""ctypes view of the hyproj C ABI (include/hyproj.h).  Argument marshalling
only: every step of the projection runs in the HIP library."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhyproj.so")

HYP_OK = 0
NOALLOC_MAX_BYTES = 128 << 20  # HYP_NOALLOC_MAX_BYTES
STATUS_OK, STATUS_MAXITER, STATUS_NONFINITE, STATUS_FLOOR, STATUS_ABORTED = 0, 1, 2, 3, 4
METHODS = {"hybrid": 0, "jacobi": 1, "pcg": 2, "cnn": 3}
PRECISIONS = {"fp32": 0, "bf16": 1}
NET_TRAIN = 1
CRITERIA = {"e1": 0, "einf": 1}
ARCHS = {"parallel": 0, "multiscale": 1, "smallscale": 2, "unet": 3}

c_i32, c_i64, c_f64, c_f32, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float, ctypes.c_void_p


class NetDesc(ctypes.Structure):
    _fields_ = [("scales", c_i32), ("channels", c_i32), ("precision", c_i32), ("flags", c_i32),
                ("arch", c_i32)]


class Grid(ctypes.Structure):
    _fields_ = [("nx", c_i32), ("ny", c_i32), ("dx", c_f64), ("dt", c_f64), ("rho0", c_f64)]


class Fields(ctypes.Structure):
    _fields_ = [("u", c_vp), ("v", c_vp), ("rho", c_vp), ("flags", c_vp), ("p", c_vp), ("p_init", c_vp),
                ("phi_ckpt", c_vp)]


class Opts(ctypes.Structure):
    _fields_ = [("method", c_i32), ("max_iters", c_i32), ("check_every", c_i32),
                ("fixed_iters", c_i32), ("omega", c_f32), ("fold_window", c_i32),
                ("checkpoint_every", c_i32), ("tile_rows", c_i32), ("variable_density", c_i32),
                ("criterion", c_i32), ("block_sweeps", c_i32)]


class Result(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("status", c_i32), ("e1_init", c_f64), ("e1_cnn", c_f64),
                ("e1_final", c_f64), ("einf_final", c_f64), ("s", c_f64),
                ("n_fluid", c_i32), ("reserved", c_i32), ("dt", c_f64)]


class Physics(ctypes.Structure):
    _fields_ = [("g", c_f64), ("rho0", c_f64), ("drho", c_f64), ("u_in", c_f64), ("cfl", c_f64)]


class State(ctypes.Structure):
    _fields_ = [("rho", c_vp), ("u", c_vp), ("v", c_vp), ("p", c_vp), ("flags", c_vp), ("xi", c_vp)]


# name -> (restype, argtypes); mirrors the declarations of include/hyproj.h
SIGNATURES = {
    "hyp_version": (c_i32, []),
    "hyp_status_str": (ctypes.c_char_p, [c_i32]),
    "hyp_create": (c_i32, [ctypes.POINTER(c_vp), ctypes.POINTER(NetDesc)]),
    "hyp_destroy": (c_i32, [c_vp]),
    "hyp_param_count": (c_i64, [c_vp]),
    "hyp_set_weights": (c_i32, [c_vp, c_vp, c_i64]),
    "hyp_workspace_size": (c_i32, [c_vp, ctypes.POINTER(Grid), ctypes.POINTER(ctypes.c_size_t)]),
    "hyp_plan": (c_i32, [c_vp, ctypes.POINTER(Grid), c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hyp_project": (c_i32, [c_vp, ctypes.POINTER(Grid), ctypes.POINTER(Fields), c_f64,
                            ctypes.POINTER(Opts), c_vp, ctypes.c_size_t, c_vp, c_vp]),
    "hyp_project_noalloc": (c_i32, [c_vp, ctypes.POINTER(Grid), ctypes.POINTER(Fields), c_f64,
                                    ctypes.POINTER(Opts), c_vp, c_vp]),
    "hyp_set_timing": (c_i32, [c_vp, c_i32]),
    "hyp_get_timing": (c_i32, [c_vp, ctypes.POINTER(c_f32)]),
    "hyp_step": (c_i32, [c_vp, ctypes.POINTER(Grid), ctypes.POINTER(Physics), ctypes.POINTER(State),
                         c_f64, ctypes.POINTER(Opts), c_vp, ctypes.c_size_t, c_vp, c_vp]),
    "hyp_advect": (c_i32, [c_vp, ctypes.POINTER(Grid), ctypes.POINTER(Physics), ctypes.POINTER(State),
                           c_vp, ctypes.c_size_t, c_vp]),
    "hyp_project_backward": (c_i32, [c_vp, ctypes.POINTER(Grid), c_i32, c_f32, c_f64, c_i32, c_vp,
                                     c_vp, c_vp, c_vp, c_vp, ctypes.c_size_t, c_vp]),
    "hyp_batch_workspace_size": (c_i32, [c_vp, c_i32, c_vp, ctypes.POINTER(ctypes.c_size_t)]),
    "hyp_batch_create": (c_i32, [c_vp, c_i32, c_vp, c_vp, c_vp, c_vp, ctypes.POINTER(Opts), c_vp,
                                 ctypes.c_size_t, ctypes.POINTER(c_vp)]),
    "hyp_batch_project": (c_i32, [c_vp, c_vp, c_vp]),
    "hyp_batch_step": (c_i32, [c_vp, c_vp, c_vp]),
    "hyp_batch_capture": (c_i32, [c_vp, c_vp, c_vp]),
    "hyp_batch_launch": (c_i32, [c_vp, c_vp]),
    "hyp_batch_destroy": (c_i32, [c_vp]),
    "hyp_adam": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, c_f32, c_f32, c_f32, c_f32, c_vp]),
}

_LIB = None


class HypError(RuntimeError):
    def __init__(self, fn, code):
        msg = lib().hyp_status_str(code).decode() if _LIB is not None else str(code)
        super().__init__(f"{fn} failed: {msg} ({code})")
        self.code = code


def lib():
    """Load the in-tree HIP library; fail loudly when it is not built."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"hyproj HIP library not found at {LIB_PATH}; build it with "
                "`python -m paper_2109_09363_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = L
    return _LIB


def check(fn, code):
    if code != HYP_OK:
        raise HypError(fn, code)
