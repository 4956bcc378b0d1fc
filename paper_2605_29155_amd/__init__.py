"""Batched differentiable MPC layer (CA-AC-MPC's CA-DiffMPC) on MI355X.

Thin ctypes binding over the C ABI in include/dmpc.h (libdmpc.so, built for
gfx950 by paper_2605_29155_amd/build.py).  This module only marshals
arguments: every step of the forward solve and of the backward runs in the
HIP kernels.  There is no CPU fallback: without the built library every call
raises.

PyTorch provides device memory and the stream; tensors are float32 on the GPU,
instance-major: x0 [B,13], Q [B,T,17] (diagonal) or [B,T,153] (packed upper
triangle), p [B,T,17], u_lo/u_hi [B,4], T [B] int32 or None.
"""
import ctypes as C
import os

from . import build as _build

NX, NU, NZ, NPACK = 13, 4, 17, 153
COST_DIAG, COST_DENSE = 0, 1
NEED_GRAD, PLAIN, LPT, TUNED, TPAR, F64, F64_REDO = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40
ST_CONVERGED, ST_MAXITER, ST_NONFINITE, ST_FP64, ST_QPMAXITER, ST_REGULARIZED = 0x1, 0x2, 0x4, 0x8, 0x10, 0x20
ST_F64_REDONE = 0x40
ITERS_SHIFT = 8
ALPHA_NONE = 255
ERRORS = {-1: "EINVAL", -2: "EUNSUPPORTED", -3: "EHIP", -4: "EWORKSPACE"}


class QuadParams(C.Structure):
    _fields_ = [(n, C.c_float) for n in ("mass", "Jxx", "Jyy", "Jzz", "arm", "kappa", "dt", "g")]


class Config(C.Structure):
    _fields_ = [("B", C.c_int32), ("T_max", C.c_int32), ("cost_kind", C.c_int32), ("max_iter", C.c_int32),
                ("tol_du", C.c_float), ("ckpt_every", C.c_int32), ("fp64_pivot", C.c_float),
                ("flags", C.c_uint32)]


class LaunchChoice(C.Structure):
    _fields_ = [("plain", C.c_int32), ("lpt", C.c_int32), ("waves_per_simd", C.c_int32), ("grid_mode", C.c_int32),
                ("ms", C.c_float), ("inst_per_wave", C.c_int32)]

    def __init__(self, plain=0, lpt=0, waves_per_simd=1, grid_mode=0, ms=0.0, inst_per_wave=4):
        super().__init__(plain, lpt, waves_per_simd, grid_mode, ms, inst_per_wave)

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class DMPCError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise DMPCError("libdmpc.so is not built (run paper_2605_29155_amd/build.py); "
                            "there is no fallback path")
        # Streams and device pointers come from PyTorch, so the library must
        # bind to the HIP runtime PyTorch loaded (PyTorch ships its own copy
        # under the same soname): import torch first, then load the library.
        import torch  # noqa: F401
        L = C.CDLL(_build.LIB)
        vp, sz, i32 = C.c_void_p, C.c_size_t, C.c_int
        L.dmpc_create.argtypes = [C.POINTER(vp), i32]
        L.dmpc_destroy.argtypes = [vp]
        L.dmpc_validate.argtypes = [C.POINTER(Config)]
        L.dmpc_workspace_bytes.argtypes = [C.POINTER(Config)]
        L.dmpc_workspace_bytes.restype = sz
        L.dmpc_forward.argtypes = [vp, C.POINTER(Config), QuadParams] + [vp] * 10 + [vp, sz, vp, vp]
        L.dmpc_forward_noalloc.argtypes = [vp, C.POINTER(Config), QuadParams] + [vp] * 12
        L.dmpc_backward.argtypes = [vp, C.POINTER(Config), QuadParams] + [vp] * 5 + [sz] + [vp] * 6 + [vp]
        L.dmpc_last_launch_count.argtypes = [vp]
        L.dmpc_autotune.argtypes = [vp, C.POINTER(Config), QuadParams] + [vp] * 10 + [vp, sz, vp, C.POINTER(LaunchChoice)]
        L.dmpc_mpc_step.argtypes = [vp, C.POINTER(Config), QuadParams] + [vp] * 6
        L.dmpc_set_tuned.argtypes = [vp, C.POINTER(Config), i32, C.POINTER(LaunchChoice)]
        L.dmpc_get_tuned.argtypes = [vp, C.POINTER(Config), i32, C.POINTER(LaunchChoice)]
        L.dmpc_last_launch_choice.argtypes = [vp, C.POINTER(LaunchChoice)]
        L.dmpc_tuned_save.argtypes = [vp, C.c_char_p]
        L.dmpc_tuned_load.argtypes = [vp, C.c_char_p]
        L.dmpc_capture_begin.argtypes = [vp, vp]
        L.dmpc_capture_end.argtypes = [vp, vp, C.POINTER(vp)]
        L.dmpc_graph_launch.argtypes = [vp, vp, vp]
        L.dmpc_graph_destroy.argtypes = [vp, vp]
        L.dmpc_last_error.argtypes = [vp]
        L.dmpc_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def quad_params(d):
    return QuadParams(*[float(d[k]) for k in ("mass", "Jxx", "Jyy", "Jzz", "arm", "kappa", "dt", "g")])


def make_config(B, T_max, cost_kind=COST_DIAG, max_iter=5, tol_du=0.0, flags=0, fp64_pivot=1e-6, ckpt_every=0):
    return Config(int(B), int(T_max), int(cost_kind), int(max_iter), float(tol_du), int(ckpt_every),
                  float(fp64_pivot), int(flags))


def validate(cfg):
    return lib().dmpc_validate(C.byref(cfg))


def workspace_bytes(cfg):
    return int(lib().dmpc_workspace_bytes(C.byref(cfg)))


def _ptr(t, dtype="float32"):
    """Device pointer of a dense tensor; the C ABI reads plain row-major
    buffers, so strided views and host tensors are rejected."""
    if t is None:
        return None
    if t.device.type != "cuda":
        raise DMPCError("expected a device tensor, got one on %s" % t.device)
    if not t.is_contiguous():
        raise DMPCError("expected a contiguous tensor of shape %s" % (tuple(t.shape),))
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise DMPCError("expected %s, got %s" % (dtype, t.dtype))
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


class Handle:
    """One dmpc handle per device."""

    def __init__(self, device=0):
        self._h = C.c_void_p()
        rc = lib().dmpc_create(C.byref(self._h), int(device))
        if rc != 0:
            raise DMPCError("dmpc_create: %s" % lib().dmpc_last_error(None).decode())
        self.device = device

    def check(self, rc, what):
        if rc != 0:
            raise DMPCError("%s: %s (%s)" % (what, ERRORS.get(rc, rc), lib().dmpc_last_error(self._h).decode()))

    def launch_count(self):
        return lib().dmpc_last_launch_count(self._h)

    def __del__(self):
        try:
            if self._h:
                lib().dmpc_destroy(self._h)
        except Exception:
            pass


def alloc_workspace(cfg, device):
    """Device workspace of dmpc_workspace_bytes(cfg), 256-byte aligned."""
    import torch
    n = workspace_bytes(cfg)
    if n == 0:
        raise DMPCError("invalid configuration")
    buf = torch.empty(n + 256, dtype=torch.uint8, device=device)
    off = (-buf.data_ptr()) % 256
    return buf[off:off + n]


def forward_raw(h, cfg, params, x0, Q, p, u_lo, u_hi, T, u_out, x_out, status, ws, dlog=None, stream=None,
                u_init=None):
    """u_init: [B][T_max][4] warm start of the first rollout (None: hover)."""
    rc = lib().dmpc_forward(h._h, C.byref(cfg), params, _ptr(x0), _ptr(Q), _ptr(p), _ptr(u_lo), _ptr(u_hi), _ptr(T, "int32"),
                            _ptr(u_init), _ptr(u_out), _ptr(x_out), _ptr(status, "int32"), _ptr(ws, "uint8"),
                            ws.numel() if ws is not None else 0, _ptr(dlog, "uint8"), _stream(stream))
    h.check(rc, "dmpc_forward")


NOALLOC_WORKSPACE_BYTES = 64 << 20  # DMPC_NOALLOC_WORKSPACE_BYTES


def forward_noalloc(h, cfg, params, x0, Q, p, u_lo, u_hi, T, u_out, x_out, status, dlog=None, stream=None,
                    u_init=None):
    """dmpc_forward on the library's static workspace (no caller
    workspace, nothing allocated); forward only, and calls on one device
    must not overlap."""
    rc = lib().dmpc_forward_noalloc(h._h, C.byref(cfg), params, _ptr(x0), _ptr(Q), _ptr(p), _ptr(u_lo), _ptr(u_hi),
                                    _ptr(T, "int32"), _ptr(u_init), _ptr(u_out), _ptr(x_out), _ptr(status, "int32"),
                                    _ptr(dlog, "uint8"), _stream(stream))
    h.check(rc, "dmpc_forward_noalloc")


def autotune(h, cfg, params, x0, Q, p, u_lo, u_hi, T, u_out, x_out, status, ws, stream=None, u_init=None):
    """Time every launch choice on these inputs and store the fastest on the
    handle for this shape (synchronises the stream).  Returns the choice."""
    c = LaunchChoice()
    rc = lib().dmpc_autotune(h._h, C.byref(cfg), params, _ptr(x0), _ptr(Q), _ptr(p), _ptr(u_lo), _ptr(u_hi),
                             _ptr(T, "int32"), _ptr(u_init), _ptr(u_out), _ptr(x_out), _ptr(status, "int32"), _ptr(ws, "uint8"),
                             ws.numel(), _stream(stream), C.byref(c))
    h.check(rc, "dmpc_autotune")
    return c


def set_tuned(h, cfg, has_T, choice):
    h.check(lib().dmpc_set_tuned(h._h, C.byref(cfg), int(bool(has_T)), C.byref(choice)), "dmpc_set_tuned")


def get_tuned(h, cfg, has_T):
    c = LaunchChoice()
    rc = lib().dmpc_get_tuned(h._h, C.byref(cfg), int(bool(has_T)), C.byref(c))
    return None if rc != 0 else c


def tuned_save(h, path):
    """Write the handle's tuned launch choices to path; returns their number."""
    n = lib().dmpc_tuned_save(h._h, os.fsencode(path))
    if n < 0:
        h.check(n, "dmpc_tuned_save")
    return n


def tuned_load(h, path):
    """Add the choices saved in path for this device's architecture; returns
    how many were taken."""
    n = lib().dmpc_tuned_load(h._h, os.fsencode(path))
    if n < 0:
        h.check(n, "dmpc_tuned_load")
    return n


def last_launch_choice(h):
    c = LaunchChoice()
    h.check(lib().dmpc_last_launch_choice(h._h, C.byref(c)), "dmpc_last_launch_choice")
    return c


def mpc_step(h, cfg, params, T, x_state, u_star, u_warm=None, u_applied=None, stream=None):
    """One receding-horizon step on the device: x_state <- RK4(x_state,
    u_star[:, 0]) in place, u_applied <- u_star[:, 0], u_warm <- u_star
    shifted by one stage (last stage repeated; may be u_star itself)."""
    rc = lib().dmpc_mpc_step(h._h, C.byref(cfg), params, _ptr(T, "int32"), _ptr(x_state), _ptr(u_star),
                             _ptr(u_warm), _ptr(u_applied), _stream(stream))
    h.check(rc, "dmpc_mpc_step")


def backward_raw(h, cfg, params, Q, p, u_lo, u_hi, ws, grad_u, grad_x, grad_Q, grad_p, grad_x0, stream=None,
                 grad_dyn=None):
    """params, Q, p, u_lo, u_hi: the forward's inputs (read with
    checkpointing, and params, Q, p with grad_dyn; may be None otherwise).
    grad_dyn: [B, 8] output, dL/d(mass, Jxx, Jyy, Jzz, arm, kappa, dt, g)
    per instance, or None."""
    rc = lib().dmpc_backward(h._h, C.byref(cfg), params if params is not None else QuadParams(),
                             _ptr(Q), _ptr(p), _ptr(u_lo), _ptr(u_hi), _ptr(ws, "uint8"), ws.numel(),
                             _ptr(grad_u), _ptr(grad_x), _ptr(grad_Q), _ptr(grad_p), _ptr(grad_x0), _ptr(grad_dyn),
                             _stream(stream))
    h.check(rc, "dmpc_backward")


def capture_begin(h, stream=None):
    h.check(lib().dmpc_capture_begin(h._h, _stream(stream)), "dmpc_capture_begin")


def capture_end(h, stream=None):
    g = C.c_void_p()
    h.check(lib().dmpc_capture_end(h._h, _stream(stream), C.byref(g)), "dmpc_capture_end")
    return g


def graph_launch(h, g, stream=None):
    h.check(lib().dmpc_graph_launch(h._h, g, _stream(stream)), "dmpc_graph_launch")


def graph_destroy(h, g):
    h.check(lib().dmpc_graph_destroy(h._h, g), "dmpc_graph_destroy")


def _make_function():
    import torch

    class DMPCFunction(torch.autograd.Function):
        """u*, x*, status = DMPCFunction.apply(x0, Q, p, u_lo, u_hi, T, dyn, layer).

        Differentiable in x0, Q and p (Sec. IV after eq. (3)) and, when dyn
        (the eight model constants as a tensor) is given, in dyn: its gradient
        is the batch sum of the per-instance dL/dtheta.  The backward reuses
        the stage factors the forward stored in its workspace."""

        @staticmethod
        def forward(ctx, x0, Q, p, u_lo, u_hi, T, dyn, layer):
            # the C ABI reads dense row-major float32 buffers
            x0, Q, p, u_lo, u_hi = (a.detach().float().contiguous() for a in (x0, Q, p, u_lo, u_hi))
            if T is not None:
                T = T.to(torch.int32).contiguous()
            # the constants are passed by value: a tensor on the GPU costs one synchronisation here
            params = layer.params if dyn is None else QuadParams(*dyn.detach().double().cpu().reshape(8).tolist())
            B, Tm = p.shape[0], p.shape[1]
            want_dyn = dyn is not None and ctx.needs_input_grad[6]
            need = any(ctx.needs_input_grad[:3]) or want_dyn
            cfg = layer.config(B, Tm, need_grad=need)
            ws = alloc_workspace(cfg, p.device)
            u = torch.empty(B, Tm, NU, device=p.device, dtype=torch.float32)
            x = torch.empty(B, Tm, NX, device=p.device, dtype=torch.float32)
            st = torch.empty(B, device=p.device, dtype=torch.int32)
            if layer.autotune and get_tuned(layer.handle, cfg, T is not None) is None:
                autotune(layer.handle, cfg, params, x0, Q, p, u_lo, u_hi, T, u, x, st, ws)
                if layer.tune_file:
                    tuned_save(layer.handle, layer.tune_file)
            else:
                forward_raw(layer.handle, cfg, params, x0, Q, p, u_lo, u_hi, T, u, x, st, ws)
            ctx.cfg, ctx.ws, ctx.layer, ctx.params = cfg, ws, layer, params
            # the checkpointed backward recomputes stage factors from the inputs,
            # and dL/dtheta reads the cost
            ctx.inputs = (Q, p, u_lo, u_hi) if (cfg.ckpt_every > 0 or want_dyn) else (None,) * 4
            ctx.shapes = (x0.shape, Q.shape, p.shape)
            ctx.want_dyn = want_dyn
            ctx.dyn_meta = None if dyn is None else (dyn.shape, dyn.dtype, dyn.device)
            ctx.mark_non_differentiable(st)
            return u, x, st

        @staticmethod
        def backward(ctx, gu, gx, _gst):
            sx0, sQ, sp = ctx.shapes
            dev = ctx.ws.device
            gu = torch.zeros(sp[0], sp[1], NU, device=dev) if gu is None else gu.contiguous().float()
            gx = None if gx is None else gx.contiguous().float()
            gQ = torch.empty(sQ, device=dev, dtype=torch.float32)
            gp = torch.empty(sp, device=dev, dtype=torch.float32)
            gx0 = torch.empty(sx0, device=dev, dtype=torch.float32)
            gd = torch.empty(sp[0], 8, device=dev, dtype=torch.float32) if ctx.want_dyn else None
            backward_raw(ctx.layer.handle, ctx.cfg, ctx.params, *ctx.inputs, ctx.ws, gu, gx, gQ, gp, gx0,
                         grad_dyn=gd)
            gdyn = None
            if gd is not None:
                shape, dtype, ddev = ctx.dyn_meta
                gdyn = gd.double().sum(0).to(device=ddev, dtype=dtype).reshape(shape)
            return gx0, gQ, gp, None, None, None, gdyn, None

    return DMPCFunction


_function = None


def DMPCFunction():
    """The module-level autograd.Function (defined once)."""
    global _function
    if _function is None:
        _function = _make_function()
    return _function


class DMPCLayer:
    """Callable layer: (x0, Q, p, u_lo, u_hi, T=None, dyn=None) -> (u*, x*, status).

    dyn: optional tensor of the eight model constants (mass, Jxx, Jyy, Jzz,
    arm, kappa, dt, g) used instead of the layer's; when it requires grad,
    the backward returns dL/d(dyn) (the batch sum of dL/dtheta)."""

    def __init__(self, params, max_iter=5, tol_du=0.0, cost_kind=COST_DIAG, plain=False, lpt=True,
                 fp64_pivot=1e-6, ckpt_every=0, autotune=False, tpar=False, device=0, tune_file=None,
                 fp64=False, fp64_redo=False):
        """autotune: on the first call for a shape, time the launch choices
        (dmpc_autotune) and use the fastest for that shape from then on.
        tune_file: with autotune, a file of saved launch choices: read at
        construction if it exists, rewritten after each new tuning, so a shape
        is tuned once per machine.
        tpar: per-launch form with the time-parallel Riccati (small B, long T).
        fp64: the FP64 form (DMPC_F64): dynamics, linearisation, line search
        and stored trajectories in double, for long unconverged runs whose
        iterate is sensitive to FP32 rounding.
        fp64_redo: the FP32 form, with the instances whose control block had
        a pivot below fp64_pivot solved again in the FP64 form (DMPC_F64_REDO)."""
        self.handle = Handle(device)
        self.autotune = autotune
        self.tune_file = tune_file
        if autotune and tune_file and os.path.exists(tune_file):
            tuned_load(self.handle, tune_file)
        self.params = quad_params(params) if isinstance(params, dict) else params
        self.max_iter, self.tol_du, self.cost_kind = max_iter, tol_du, cost_kind
        self.plain, self.lpt, self.fp64_pivot, self.ckpt_every = plain, lpt, fp64_pivot, ckpt_every
        self.tpar = tpar
        self.fp64 = fp64
        self.fp64_redo = fp64_redo

    def config(self, B, T_max, need_grad=True):
        flags = (NEED_GRAD if need_grad else 0) | (PLAIN if self.plain else 0) | (LPT if self.lpt else 0)
        flags |= TUNED if self.autotune else 0
        flags |= TPAR if self.tpar else 0
        flags |= F64 if self.fp64 else 0
        flags |= F64_REDO if self.fp64_redo else 0
        return make_config(B, T_max, self.cost_kind, self.max_iter, self.tol_du, flags, self.fp64_pivot,
                           self.ckpt_every)

    def __call__(self, x0, Q, p, u_lo, u_hi, T=None, dyn=None):
        return DMPCFunction().apply(x0, Q, p, u_lo, u_hi, T, dyn, self)
