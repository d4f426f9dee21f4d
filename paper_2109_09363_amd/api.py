"""Python binding of the hyproj C ABI: torch tensors in, raw device pointers
and the current HIP stream out.  PyTorch supplies device memory and streams
only; the projection itself runs in the HIP library."""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass
class ProjectionResult:
    iters: int
    status: int
    e1_init: float
    e1_cnn: float
    e1_final: float
    einf_final: float
    s: float
    n_fluid: int
    dt: float


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor of shape {shape}, "
                         f"got {t.dtype} {tuple(t.shape)}")


class Projector:
    """One context + workspace for a grid shape (and optionally a network).

    The workspace is a caller-owned torch uint8 tensor; the library allocates
    no device memory."""

    def __init__(self, nx: int, ny: int, dx: float, dt: float = 1.0, rho0: float = 1.0,
                 scales: int = 0, channels: int = 0, precision: str = "fp32", device=None,
                 train: bool = False, arch: str = "parallel"):
        self.lib = L.lib()
        self.nx, self.ny = int(nx), int(ny)
        self.grid = L.Grid(self.nx, self.ny, float(dx), float(dt), float(rho0))
        self.device = torch.device("cuda" if device is None else device)
        ctx = ctypes.c_void_p()
        desc = None
        if arch not in L.ARCHS:
            raise ValueError(f"arch must be one of {sorted(L.ARCHS)}")
        if arch != "parallel":
            scales = 5 if arch == "unet" else 3  # the paper's networks: fixed scales
        if scales > 0:
            desc = L.NetDesc(int(scales), int(channels), L.PRECISIONS[precision],
                             L.NET_TRAIN if train else 0, L.ARCHS[arch])
        L.check("hyp_create", self.lib.hyp_create(ctypes.byref(ctx), ctypes.byref(desc) if desc else None))
        self.ctx = ctx
        self.scales, self.channels, self.precision = scales, channels, precision
        self.arch = arch
        nbytes = ctypes.c_size_t()
        L.check("hyp_workspace_size",
                self.lib.hyp_workspace_size(self.ctx, ctypes.byref(self.grid), ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.res = torch.zeros(ctypes.sizeof(L.Result), dtype=torch.uint8, device=self.device)
        self.params = None
        self.planned = False

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                self.lib.hyp_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return int(self.lib.hyp_param_count(self.ctx))

    def set_dt(self, dt: float):
        self.grid.dt = float(dt)

    def set_weights(self, params: torch.Tensor):
        _need(params, torch.float32, (self.param_count,), "params")
        L.check("hyp_set_weights", self.lib.hyp_set_weights(self.ctx, _ptr(params), params.numel()))
        self.params = params  # keep alive: the library reads it at every call

    def plan(self, flags: torch.Tensor):
        _need(flags, torch.uint8, (self.ny, self.nx), "flags")
        L.check("hyp_plan", self.lib.hyp_plan(self.ctx, ctypes.byref(self.grid), _ptr(flags),
                                              _ptr(self.ws), self.ws.numel(), _stream()))
        self.planned = True

    def project_async(self, u, v, flags, p, threshold: float, method: str = "hybrid",
                      max_iters: int = 200000, check_every: int = 8, fixed_iters: int = 0,
                      omega: float = 1.0, rho=None, p_init=None, fold_window: int = 0,
                      checkpoint_every: int = 0, phi_ckpt=None, tile_rows: int = 0,
                      variable_density: bool = False, criterion: str = "e1", block_sweeps: int = 0):
        """Enqueue one projection on the current stream; u, v corrected in
        place, p written.  Read the result with `result()` after a sync.
        With fixed_iters and checkpoint_every > 0, phi_ckpt (n, ny, nx) float32
        receives the Jacobi iterate after every checkpoint_every sweeps.
        variable_density keeps rho (required then) inside the operator;
        criterion "einf" stops on max |div u| instead of the mean."""
        nx, ny = self.nx, self.ny
        _need(u, torch.float32, (ny, nx + 1), "u")
        _need(v, torch.float32, (ny + 1, nx), "v")
        _need(flags, torch.uint8, (ny, nx), "flags")
        _need(p, torch.float32, (ny, nx), "p")
        if rho is not None:
            _need(rho, torch.float32, (ny, nx), "rho")
        elif variable_density:
            raise ValueError("variable_density needs rho")
        if p_init is not None:
            _need(p_init, torch.float32, (ny, nx), "p_init")
        if phi_ckpt is not None:
            if checkpoint_every <= 0 or fixed_iters <= 0:
                raise ValueError("phi_ckpt needs checkpoint_every > 0 and fixed_iters > 0")
            _need(phi_ckpt, torch.float32, (fixed_iters // checkpoint_every, ny, nx), "phi_ckpt")
        if not self.planned:
            raise RuntimeError("call plan(flags) before project")
        f = L.Fields(_ptr(u), _ptr(v), _ptr(rho), _ptr(flags), _ptr(p), _ptr(p_init), _ptr(phi_ckpt))
        o = L.Opts(L.METHODS[method], int(max_iters), int(check_every), int(fixed_iters),
                   float(omega), int(fold_window), int(checkpoint_every), int(tile_rows),
                   1 if variable_density else 0, L.CRITERIA[criterion], int(block_sweeps))
        L.check("hyp_project", self.lib.hyp_project(
            self.ctx, ctypes.byref(self.grid), ctypes.byref(f), float(threshold), ctypes.byref(o),
            _ptr(self.ws), self.ws.numel(), _stream(), _ptr(self.res)))

    def project_noalloc_async(self, u, v, flags, p, threshold: float, method: str = "hybrid",
                              max_iters: int = 200000, check_every: int = 8, fixed_iters: int = 0,
                              omega: float = 1.0, rho=None, p_init=None, fold_window: int = 0,
                              tile_rows: int = 0, variable_density: bool = False,
                              criterion: str = "e1"):
        """project_async without the context's workspace: the library plans
        `flags` and projects in its static per-GPU array (hyp_project_noalloc;
        grids whose workspace exceeds NOALLOC_MAX_BYTES are rejected).  Calls
        that overlap on one GPU race on that array."""
        nx, ny = self.nx, self.ny
        _need(u, torch.float32, (ny, nx + 1), "u")
        _need(v, torch.float32, (ny + 1, nx), "v")
        _need(flags, torch.uint8, (ny, nx), "flags")
        _need(p, torch.float32, (ny, nx), "p")
        if rho is not None:
            _need(rho, torch.float32, (ny, nx), "rho")
        elif variable_density:
            raise ValueError("variable_density needs rho")
        if p_init is not None:
            _need(p_init, torch.float32, (ny, nx), "p_init")
        f = L.Fields(_ptr(u), _ptr(v), _ptr(rho), _ptr(flags), _ptr(p), _ptr(p_init), None)
        o = L.Opts(L.METHODS[method], int(max_iters), int(check_every), int(fixed_iters),
                   float(omega), int(fold_window), 0, int(tile_rows),
                   1 if variable_density else 0, L.CRITERIA[criterion])
        L.check("hyp_project_noalloc", self.lib.hyp_project_noalloc(
            self.ctx, ctypes.byref(self.grid), ctypes.byref(f), float(threshold), ctypes.byref(o),
            _stream(), _ptr(self.res)))

    def advect_async(self, rho, u, v, xi, g: float, drho: float, u_in: float = 1.0,
                     cfl: float = 0.5):
        """Enqueue the advection + force half step: u, v become u*."""
        nx, ny = self.nx, self.ny
        _need(rho, torch.float32, (ny, nx), "rho")
        _need(u, torch.float32, (ny, nx + 1), "u")
        _need(v, torch.float32, (ny + 1, nx), "v")
        _need(xi, torch.float32, (nx,), "xi")
        if not self.planned:
            raise RuntimeError("call plan(flags) before advect")
        ph = L.Physics(float(g), float(self.grid.rho0), float(drho), float(u_in), float(cfl))
        st = L.State(_ptr(rho), _ptr(u), _ptr(v), None, None, _ptr(xi))
        L.check("hyp_advect", self.lib.hyp_advect(self.ctx, ctypes.byref(self.grid), ctypes.byref(ph),
                                                  ctypes.byref(st), _ptr(self.ws), self.ws.numel(),
                                                  _stream()))

    def backward_async(self, sweeps: int, omega: float = 1.0, scale: float = 1.0, du=None, dv=None,
                       dparams=None, loss=None, accumulate: bool = False):
        """Gradient of scale * sum_F r^2 after the last forward (hybrid with
        fixed_iters = sweeps, or method 'cnn' for sweeps = 0)."""
        nx, ny = self.nx, self.ny
        if du is not None:
            _need(du, torch.float32, (ny, nx + 1), "du")
        if dv is not None:
            _need(dv, torch.float32, (ny + 1, nx), "dv")
        if dparams is not None:
            _need(dparams, torch.float32, (self.param_count,), "dparams")
        if loss is not None:
            _need(loss, torch.float64, (1,), "loss")
        L.check("hyp_project_backward", self.lib.hyp_project_backward(
            self.ctx, ctypes.byref(self.grid), int(sweeps), float(omega), float(scale),
            1 if accumulate else 0, _ptr(du), _ptr(dv), _ptr(dparams), _ptr(loss), _ptr(self.ws),
            self.ws.numel(), _stream()))

    def set_timing(self, enable: bool = True):
        L.check("hyp_set_timing", self.lib.hyp_set_timing(self.ctx, 1 if enable else 0))

    def timing(self) -> dict:
        """Phase times (ms) of the last call: advection, divergence + CNN
        (t_inf), solver, correction, total."""
        arr = (ctypes.c_float * 5)()
        L.check("hyp_get_timing", self.lib.hyp_get_timing(self.ctx, arr))
        return dict(advect=arr[0], inference=arr[1], solver=arr[2], correct=arr[3], total=arr[4])

    def result(self) -> ProjectionResult:
        raw = bytes(self.res.cpu().numpy().tobytes())
        r = L.Result.from_buffer_copy(raw)
        return ProjectionResult(r.iters, r.status, r.e1_init, r.e1_cnn, r.e1_final,
                                r.einf_final, r.s, r.n_fluid, r.dt)

    def step_async(self, rho, u, v, flags, p, xi, threshold: float, g: float, drho: float,
                   u_in: float = 1.0, cfl: float = 0.5, method: str = "hybrid",
                   max_iters: int = 200000, check_every: int = 8, fixed_iters: int = 0,
                   omega: float = 1.0, fold_window: int = 0, variable_density: bool = False,
                   criterion: str = "e1", tile_rows: int = 0, block_sweeps: int = 0):
        """Enqueue one full time step (advection, buoyancy, inflow, projection)
        on the current stream.  rho, u, v advance in place; p is written.
        variable_density projects with the advected density in the operator."""
        nx, ny = self.nx, self.ny
        _need(rho, torch.float32, (ny, nx), "rho")
        _need(u, torch.float32, (ny, nx + 1), "u")
        _need(v, torch.float32, (ny + 1, nx), "v")
        _need(flags, torch.uint8, (ny, nx), "flags")
        _need(p, torch.float32, (ny, nx), "p")
        _need(xi, torch.float32, (nx,), "xi")
        if not self.planned:
            raise RuntimeError("call plan(flags) before step")
        ph = L.Physics(float(g), float(self.grid.rho0), float(drho), float(u_in), float(cfl))
        st = L.State(_ptr(rho), _ptr(u), _ptr(v), _ptr(p), _ptr(flags), _ptr(xi))
        o = L.Opts(L.METHODS[method], int(max_iters), int(check_every), int(fixed_iters),
                   float(omega), int(fold_window), 0, int(tile_rows), 1 if variable_density else 0,
                   L.CRITERIA[criterion], int(block_sweeps))
        L.check("hyp_step", self.lib.hyp_step(
            self.ctx, ctypes.byref(self.grid), ctypes.byref(ph), ctypes.byref(st), float(threshold),
            ctypes.byref(o), _ptr(self.ws), self.ws.numel(), _stream(), _ptr(self.res)))


class Batch:
    """Many plumes of uneven sizes projected (or stepped) together: one launch
    per phase over all instances and one persistent Jacobi launch.
    `instances` is a list of dicts with keys nx, ny, dx, flags, u, v, p and
    optionally rho, xi, dt, rho0, threshold, and the instance's physics g,
    drho, u_in, cfl (needed by step_async / capture; each plume its own)."""

    def __init__(self, instances, threshold: float = 1e-3, method: str = "hybrid",
                 params=None, scales: int = 0, channels: int = 0, precision: str = "fp32",
                 max_iters: int = 200000, omega: float = 1.0, device=None,
                 variable_density: bool = False, tile_rows: int = 0, check_every: int = 8):
        self.lib = L.lib()
        self.device = torch.device("cuda" if device is None else device)
        ctx = ctypes.c_void_p()
        desc = L.NetDesc(int(scales), int(channels), L.PRECISIONS[precision], 0) if scales > 0 else None
        L.check("hyp_create", self.lib.hyp_create(ctypes.byref(ctx), ctypes.byref(desc) if desc else None))
        self.ctx = ctx
        self.n = len(instances)
        self.inst = instances
        if params is not None:
            _need(params, torch.float32, (int(self.lib.hyp_param_count(self.ctx)),), "params")
            L.check("hyp_set_weights", self.lib.hyp_set_weights(self.ctx, _ptr(params), params.numel()))
            self.params = params
        G = (L.Grid * self.n)()
        S = (L.State * self.n)()
        T = (ctypes.c_double * self.n)()
        have_phys = all("g" in d for d in instances)
        PH = (L.Physics * self.n)() if have_phys else None
        for i, d in enumerate(instances):
            nx, ny = int(d["nx"]), int(d["ny"])
            G[i] = L.Grid(nx, ny, float(d["dx"]), float(d.get("dt", 1.0)), float(d.get("rho0", 1.0)))
            _need(d["u"], torch.float32, (ny, nx + 1), "u")
            _need(d["v"], torch.float32, (ny + 1, nx), "v")
            _need(d["p"], torch.float32, (ny, nx), "p")
            _need(d["flags"], torch.uint8, (ny, nx), "flags")
            if d.get("rho") is not None:
                _need(d["rho"], torch.float32, (ny, nx), "rho")
            elif variable_density:
                raise ValueError("variable_density needs rho for every instance")
            if d.get("xi") is not None:
                _need(d["xi"], torch.float32, (nx,), "xi")
            S[i] = L.State(_ptr(d.get("rho")), _ptr(d["u"]), _ptr(d["v"]), _ptr(d["p"]),
                           _ptr(d["flags"]), _ptr(d.get("xi")))
            T[i] = float(d.get("threshold", threshold))
            if have_phys:
                PH[i] = L.Physics(float(d["g"]), float(d.get("rho0", 1.0)), float(d.get("drho", 0.01)),
                                  float(d.get("u_in", 1.0)), float(d.get("cfl", 0.5)))
        self.has_physics = have_phys
        self._grids, self._states, self._thr, self._phys = G, S, T, PH
        nbytes = ctypes.c_size_t()
        L.check("hyp_batch_workspace_size",
                self.lib.hyp_batch_workspace_size(self.ctx, self.n, G, ctypes.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.res = torch.zeros(self.n * ctypes.sizeof(L.Result), dtype=torch.uint8, device=self.device)
        o = L.Opts(L.METHODS[method], int(max_iters), int(check_every), 0, float(omega), 0, 0, int(tile_rows),
                   1 if variable_density else 0, 0)
        b = ctypes.c_void_p()
        torch.cuda.synchronize()
        L.check("hyp_batch_create", self.lib.hyp_batch_create(
            self.ctx, self.n, G, S, T, PH, ctypes.byref(o), _ptr(self.ws), self.ws.numel(),
            ctypes.byref(b)))
        self.batch = b

    def __del__(self):
        try:
            if getattr(self, "batch", None):
                self.lib.hyp_batch_destroy(self.batch)
                self.batch = None
            if getattr(self, "ctx", None):
                self.lib.hyp_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    def project_async(self):
        L.check("hyp_batch_project", self.lib.hyp_batch_project(self.batch, _stream(), _ptr(self.res)))

    def step_async(self):
        """One time step of every instance with its own physics."""
        L.check("hyp_batch_step", self.lib.hyp_batch_step(self.batch, _stream(), _ptr(self.res)))

    def capture(self):
        """Record one batched time step as a hipGraph (on a side stream)."""
        s = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            L.check("hyp_batch_capture", self.lib.hyp_batch_capture(self.batch, _stream(),
                                                                    _ptr(self.res)))
        torch.cuda.synchronize()

    def launch_async(self):
        L.check("hyp_batch_launch", self.lib.hyp_batch_launch(self.batch, _stream()))

    def results(self):
        raw = bytes(self.res.cpu().numpy().tobytes())
        sz = ctypes.sizeof(L.Result)
        out = []
        for i in range(self.n):
            r = L.Result.from_buffer_copy(raw[i * sz:(i + 1) * sz])
            out.append(ProjectionResult(r.iters, r.status, r.e1_init, r.e1_cnn, r.e1_final,
                                        r.einf_final, r.s, r.n_fluid, r.dt))
        return out


def adam_async(params, grads, m, v, step: int, lr: float = 1e-3, beta1: float = 0.9,
               beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update of FP32 device tensors on the current stream."""
    for t, name in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
        _need(t, torch.float32, tuple(params.shape), name)
    L.check("hyp_adam", L.lib().hyp_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(),
                                         int(step), float(lr), float(beta1), float(beta2), float(eps),
                                         _stream()))


class ProjectionLoss(torch.autograd.Function):
    """loss = scale * sum_F r^2 of the hybrid projection with `sweeps` fixed
    Jacobi sweeps, differentiable w.r.t. u, v and the network parameters
    through the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, u, v, params, projector, flags, sweeps, omega, scale):
        pr = projector
        pr.set_weights(params)
        uu, vv = u.detach().clone(), v.detach().clone()
        p = torch.empty((pr.ny, pr.nx), dtype=torch.float32, device=u.device)
        method = "hybrid" if sweeps > 0 else "cnn"
        pr.project_async(uu, vv, flags, p, 0.0, method=method, fixed_iters=sweeps, omega=omega)
        loss = torch.zeros(1, dtype=torch.float64, device=u.device)
        du = torch.empty_like(u)
        dv = torch.empty_like(v)
        dp = torch.empty_like(params)
        pr.backward_async(sweeps, omega, scale, du=du, dv=dv, dparams=dp, loss=loss)
        ctx.save_for_backward(du, dv, dp)
        return loss[0].to(torch.float32)

    @staticmethod
    def backward(ctx, gout):
        du, dv, dp = ctx.saved_tensors
        g = gout.to(torch.float32)
        return g * du, g * dv, g * dp, None, None, None, None, None


_CACHE: dict = {}


def project(u, v, rho, flags, threshold: float, *, dx: float, dt: float = 1.0, rho0: float = 1.0,
            method: str = "hybrid", params=None, scales: int = 0, channels: int = 0,
            precision: str = "fp32", **opts):
    """project(u, v, rho, flags, threshold) -> (p, u, v, iters).

    u, v are corrected in place (and returned); p is a new tensor.  A context
    and workspace are cached per (shape, network); the flags are planned
    again only when they differ from the last planned ones."""
    ny, nx = flags.shape
    key = (nx, ny, scales, channels, precision, u.device)
    pr = _CACHE.get(key)
    if pr is None:
        pr = Projector(nx, ny, dx, dt, rho0, scales, channels, precision, device=u.device)
        _CACHE[key] = pr
    pr.grid.dx, pr.grid.dt, pr.grid.rho0 = float(dx), float(dt), float(rho0)
    if params is not None:
        pr.set_weights(params)
    planned = getattr(pr, "_planned_flags", None)
    if planned is None or not torch.equal(planned, flags):
        pr.plan(flags)
        pr._planned_flags = flags.clone()
    p = torch.empty((ny, nx), dtype=torch.float32, device=u.device)
    pr.project_async(u, v, flags, p, threshold, method=method, rho=rho, **opts)
    res = pr.result()
    return p, u, v, res.iters
