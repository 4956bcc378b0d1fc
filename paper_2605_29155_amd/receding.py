"""Receding-horizon driver (Alg. 1/2 outer loop): at every control step the
horizon problem is solved from the current state, its first control is
applied to the plant and the horizon moves on by one stage.

The driver only chains two library calls per step on one stream:
dmpc_forward (warm-started from the shifted previous solution) and
dmpc_mpc_step (one RK4 step of the model with u*_0, and the shift).  The
plant is the quadrotor model itself; a caller with a real plant reads
`u_applied` and writes the measured state into `x` before the next step.
"""
from . import (COST_DIAG, LPT, NU, NX, PLAIN, TPAR, DMPCError, Handle, alloc_workspace, capture_begin, capture_end,
               forward_raw, graph_destroy, graph_launch, make_config, mpc_step, quad_params)


class RecedingHorizon:
    """Closed-loop MPC on B instances with horizons up to T_max.

    warm: start each solve after reset() from the previous solution shifted
    by one stage (last stage repeated); otherwise every solve starts from
    hover thrust.  With tol_du > 0 a warm start lets a solve stop after fewer
    iterations.  State, solution and warm start stay on the device."""

    def __init__(self, params, B, T_max, max_iter=5, tol_du=0.0, cost_kind=COST_DIAG, warm=True, lpt=True,
                 plain=False, tpar=False, fp64_pivot=1e-6, device=0, handle=None):
        import torch
        self.handle = handle if handle is not None else Handle(device)
        self.params = quad_params(params) if isinstance(params, dict) else params
        flags = (LPT if lpt else 0) | (PLAIN if plain else 0) | (TPAR if tpar else 0)
        self.cfg = make_config(B, T_max, cost_kind, max_iter, tol_du, flags, fp64_pivot)
        self.warm = warm
        dev = torch.device("cuda", device)
        self.ws = alloc_workspace(self.cfg, dev)
        f32 = dict(device=dev, dtype=torch.float32)
        self.x = torch.zeros(B, NX, **f32)           # plant state
        self.u = torch.zeros(B, T_max, NU, **f32)    # last solution U*
        self.x_pred = torch.zeros(B, T_max, NX, **f32)
        self.u_warm = torch.zeros(B, T_max, NU, **f32)
        self.u_applied = torch.zeros(B, NU, **f32)
        self.status = torch.zeros(B, dtype=torch.int32, device=dev)
        self._started = False
        self._graph = None

    def reset(self, x0):
        """Set the plant state; the next solve starts cold (hover thrust)."""
        self.x.copy_(x0)
        self._started = False

    def step(self, Q, p, u_lo, u_hi, T=None, stream=None, dlog=None):
        """One control step: solve from self.x, apply u*_0, shift.  Returns
        (u_applied [B,4], status [B]); both are overwritten by the next step."""
        if self._graph is not None:
            raise DMPCError("a captured step is active; use replay() or release()")
        u_init = self.u_warm if (self.warm and self._started) else None
        forward_raw(self.handle, self.cfg, self.params, self.x, Q, p, u_lo, u_hi, T, self.u, self.x_pred,
                    self.status, self.ws, dlog, stream, u_init=u_init)
        mpc_step(self.handle, self.cfg, self.params, T, self.x, self.u, self.u_warm if self.warm else None,
                 self.u_applied, stream)
        self._started = True
        return self.u_applied, self.status

    def capture(self, Q, p, u_lo, u_hi, T=None, stream=None):
        """Capture one warm-started step (forward + apply/shift) on these input
        buffers into a HIP graph; replay() then runs it with one launch call.
        The inputs are read at replay time, so update them in place.  Needs
        warm=True and one eager step() before, so that u_warm holds a shift."""
        import torch
        if not (self.warm and self._started):
            raise DMPCError("capture needs warm=True and one eager step() first")
        s = stream if stream is not None else torch.cuda.Stream(device=self.x.device)
        s.wait_stream(torch.cuda.current_stream(self.x.device))
        with torch.cuda.stream(s):
            capture_begin(self.handle, s)
            forward_raw(self.handle, self.cfg, self.params, self.x, Q, p, u_lo, u_hi, T, self.u, self.x_pred,
                        self.status, self.ws, None, s, u_init=self.u_warm)
            mpc_step(self.handle, self.cfg, self.params, T, self.x, self.u, self.u_warm, self.u_applied, s)
            self._graph = capture_end(self.handle, s)
        self._graph_stream = s
        return self._graph

    def replay(self):
        graph_launch(self.handle, self._graph, self._graph_stream)
        return self.u_applied, self.status

    def release(self):
        if self._graph is not None:
            import torch
            torch.cuda.current_stream(self.x.device).wait_stream(self._graph_stream)
            self._graph_stream.synchronize()
            graph_destroy(self.handle, self._graph)
            self._graph = None

    def __del__(self):
        try:
            self.release()
        except Exception:
            pass
