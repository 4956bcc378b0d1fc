"""ctypes binding of the FP64 CPU oracle (liboracle.so).

TEST INFRASTRUCTURE ONLY: imported by tests/, __graft_entry__.smoke() and the
CPU-baseline leg of bench.py.  The product package never imports it.

Arrays are numpy float64 (int32 / uint8 where noted), instance-major:
x0 [B,13], Q [B,T,17|153|289], p [B,T,17], lo/hi [B,4], T [B],
u [B,T,4], x [B,T,13].
"""
import ctypes as C
import os

import numpy as np

from . import build as _build

NX, NU, NZ, NPACK, NALPHA, NTHETA = 13, 4, 17, 153, 4, 8
THETA_NAMES = ("mass", "Jxx", "Jyy", "Jzz", "arm", "kappa", "dt", "g")
COST_DIAG, COST_PACKED, COST_FULL = 0, 1, 2
DYN_QUAD, DYN_AFFINE = 0, 1
ST_CONVERGED, ST_MAXITER, ST_NONFINITE, ST_QPFAIL, ST_REGULARIZED = 0x1, 0x2, 0x4, 0x10, 0x20
FREE, LOWER, UPPER = 0, 1, 2
ALPHA_NONE = 255


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("mass", "Jxx", "Jyy", "Jzz", "arm", "kappa", "dt", "g")]


class Config(C.Structure):
    _fields_ = [("B", C.c_int32), ("T_max", C.c_int32), ("cost_kind", C.c_int32), ("dyn_kind", C.c_int32),
                ("max_iter", C.c_int32), ("tol", C.c_double), ("nthreads", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        # DMPC_ORACLE_LIB lets the mutation test load a deliberately broken copy
        path = os.environ.get("DMPC_ORACLE_LIB", _build.LIB)
        if path == _build.LIB and not os.path.exists(path):
            _build.build()
        _lib = C.CDLL(path)
    return _lib


def alphas():
    """The C oracle's line-search step lengths, in the order it tries them
    (Sec. IV "Forward pass with line-search")."""
    out = np.zeros(NALPHA)
    n = lib().orc_alphas(_ptr(out))
    return tuple(float(a) for a in out[:n])


def params(mass=0.75, Jxx=2.5e-3, Jyy=2.5e-3, Jzz=4.5e-3, arm=0.15, kappa=0.01, dt=0.05, g=9.81):
    return Params(mass, Jxx, Jyy, Jzz, arm, kappa, dt, g)


def params_from(d):
    return Params(*[float(d[k]) for k in ("mass", "Jxx", "Jyy", "Jzz", "arm", "kappa", "dt", "g")])


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a, t=C.c_double):
    return None if a is None else a.ctypes.data_as(C.POINTER(t))


def dyn(P, x, u):
    out = np.zeros(NX)
    lib().orc_dyn(C.byref(P), _ptr(_d(x)), _ptr(_d(u)), _ptr(out))
    return out


def rk4(P, x, u):
    out = np.zeros(NX)
    lib().orc_rk4(C.byref(P), _ptr(_d(x)), _ptr(_d(u)), _ptr(out))
    return out


def rk4_complex_step(P, x, u, direction, h=1e-30):
    out = np.zeros(NX)
    lib().orc_rk4_complex_step(C.byref(P), _ptr(_d(x)), _ptr(_d(u)), _ptr(_d(direction)), C.c_double(h),
                               _ptr(out))
    return out


def dyn_jac(P, x, u):
    Fx, Fu = np.zeros((NX, NX)), np.zeros((NX, NU))
    lib().orc_dyn_jac(C.byref(P), _ptr(_d(x)), _ptr(_d(u)), _ptr(Fx), _ptr(Fu))
    return Fx, Fu


def rk4_jac(P, x, u):
    A, B = np.zeros((NX, NX)), np.zeros((NX, NU))
    lib().orc_rk4_jac(C.byref(P), _ptr(_d(x)), _ptr(_d(u)), _ptr(A), _ptr(B))
    return A, B


def boxqp(H, q, a, b):
    d = np.zeros(NU)
    pat = np.zeros(NU, dtype=np.int32)
    f = lib().orc_boxqp
    f.restype = C.c_uint32
    st = f(_ptr(_d(H)), _ptr(_d(q)), _ptr(_d(a)), _ptr(_d(b)), _ptr(d), _ptr(pat, C.c_int32))
    return d, pat, int(st)


def lu_solve(M, r):
    M = _d(M).copy()
    r = _d(r).copy()
    rc = lib().orc_lu_solve(C.c_int(M.shape[0]), _ptr(M), _ptr(r))
    if rc != 0:
        raise np.linalg.LinAlgError("singular")
    return r


def cost_kind_of(Q):
    w = Q.shape[-1]
    return {NZ: COST_DIAG, NPACK: COST_PACKED, NZ * NZ: COST_FULL}[w]


def _cfg(B, Tmax, cost_kind, dyn_kind, K, tol, nthreads):
    return Config(B, Tmax, cost_kind, dyn_kind, K, float(tol), max(1, int(nthreads)))


def forward(P, x0, Q, p, lo, hi, T=None, K=5, tol=0.0, affine=None, u_init=None, replay=None, nthreads=None):
    """Control-limited iLQR on a batch.  Returns a dict of outputs.

    affine = (A [B,T,13,13], Bm [B,T,13,4], r [B,T,13]) selects the affine
    dynamics; replay = (iters [B], alpha [B,K], pattern [B,K,T]) replays
    another solver's decisions, and then out["replay_viol"] [B,K,T] scores
    each replayed clamp pattern against the oracle's own stage QP (0 when it
    satisfies the QP's optimality conditions, else the smallest relative
    tolerance at which it would)."""
    x0, p, lo, hi = _d(x0), _d(p), _d(lo), _d(hi)
    Q = _d(Q)
    B, Tm = p.shape[0], p.shape[1]
    Q = Q.reshape(B, Tm, -1)
    ck = cost_kind_of(Q)
    Tarr = None if T is None else np.ascontiguousarray(T, dtype=np.int32)
    nthreads = nthreads or min(8, os.cpu_count() or 1)
    cfg = _cfg(B, Tm, ck, DYN_AFFINE if affine is not None else DYN_QUAD, K, tol, nthreads)
    Aff = Bff = rff = None
    if affine is not None:
        Aff, Bff, rff = (_d(a) for a in affine)
    ui = None if u_init is None else _d(u_init)
    ri = ra = rp = None
    if replay is not None:
        ri = np.ascontiguousarray(replay[0], dtype=np.int32)
        ra = np.ascontiguousarray(replay[1], dtype=np.uint8)
        rp = np.ascontiguousarray(replay[2], dtype=np.uint8)
        assert ra.shape == (B, K) and rp.shape == (B, K, Tm)
    out = dict(u=np.zeros((B, Tm, NU)), x=np.zeros((B, Tm, NX)), J=np.zeros(B), iters=np.zeros(B, np.int32),
               status=np.zeros(B, np.uint32), alpha=np.zeros((B, K), np.uint8),
               pattern=np.zeros((B, K, Tm), np.uint8), cand_cost=np.zeros((B, K, NALPHA)),
               replay_viol=np.zeros((B, K, Tm)))
    rc = lib().orc_forward(
        C.byref(cfg), C.byref(P), _ptr(x0), _ptr(Q), _ptr(p), _ptr(lo), _ptr(hi), _ptr(Tarr, C.c_int32),
        _ptr(Aff), _ptr(Bff), _ptr(rff), _ptr(ui), _ptr(ri, C.c_int32), _ptr(ra, C.c_uint8), _ptr(rp, C.c_uint8),
        _ptr(out["u"]), _ptr(out["x"]), _ptr(out["J"]), _ptr(out["iters"], C.c_int32),
        _ptr(out["status"], C.c_uint32), _ptr(out["alpha"], C.c_uint8), _ptr(out["pattern"], C.c_uint8),
        _ptr(out["cand_cost"]), _ptr(out["replay_viol"]))
    if rc != 0:
        raise ValueError("orc_forward rejected its arguments")
    return out


def backward(P, x0, Q, p, lo, hi, u_star, x_star, grad_u, grad_x=None, T=None, mask=None, method=0,
             affine=None, nthreads=None, dtheta=False):
    """Implicit-KKT gradients at (x*, u*).  method 0 = Riccati adjoint,
    1 = dense KKT.  Returns dict(dQ, dp, dx0), plus dtheta [B, 8] (dL/d of
    mass, Jxx, Jyy, Jzz, arm, kappa, dt, g) when dtheta is True."""
    x0, p, lo, hi = _d(x0), _d(p), _d(lo), _d(hi)
    Q = _d(Q)
    B, Tm = p.shape[0], p.shape[1]
    Q = Q.reshape(B, Tm, -1)
    ck = cost_kind_of(Q)
    Tarr = None if T is None else np.ascontiguousarray(T, dtype=np.int32)
    nthreads = nthreads or min(8, os.cpu_count() or 1)
    cfg = _cfg(B, Tm, ck, DYN_AFFINE if affine is not None else DYN_QUAD, 0, 0.0, nthreads)
    Aff = Bff = rff = None
    if affine is not None:
        Aff, Bff, rff = (_d(a) for a in affine)
    m = None if mask is None else np.ascontiguousarray(mask, dtype=np.uint8)
    gx = None if grad_x is None else _d(grad_x)
    out = dict(dQ=np.zeros_like(Q), dp=np.zeros((B, Tm, NZ)), dx0=np.zeros((B, NX)))
    if dtheta:
        out["dtheta"] = np.zeros((B, NTHETA))
    rc = lib().orc_backward(
        C.byref(cfg), C.byref(P), _ptr(x0), _ptr(Q), _ptr(p), _ptr(lo), _ptr(hi), _ptr(Tarr, C.c_int32),
        _ptr(Aff), _ptr(Bff), _ptr(rff), _ptr(_d(u_star)), _ptr(_d(x_star)), _ptr(m, C.c_uint8),
        _ptr(_d(grad_u)), _ptr(gx), C.c_int32(method), _ptr(out["dQ"]), _ptr(out["dp"]), _ptr(out["dx0"]),
        _ptr(out.get("dtheta")))
    if rc != 0:
        raise ValueError("orc_backward failed (bad arguments or singular KKT system)")
    return out


def active_mask(u, lo, hi, T=None):
    """[B,T] uint8, bit i set when control i equals a bound exactly."""
    u = np.asarray(u)
    lo = np.asarray(lo)[:, None, :]
    hi = np.asarray(hi)[:, None, :]
    act = (u == lo) | (u == hi)
    m = np.zeros(u.shape[:2], np.uint8)
    for i in range(NU):
        m |= (act[..., i].astype(np.uint8) << i)
    if T is not None:
        m[np.arange(u.shape[1])[None, :] >= np.asarray(T)[:, None]] = 0
    return m


def shift_warm_start(u, T=None):
    """Initial controls U^0 of the next receding-horizon solve built from this
    solve's U* (Alg. 1/2 outer loop with a shifted warm start): stage t takes
    stage t + 1, the last stage of each horizon repeats, stages >= T_b are 0."""
    u = np.asarray(u, np.float64)
    B, Tm = u.shape[:2]
    Tb = np.full(B, Tm) if T is None else np.asarray(T)
    out = np.zeros_like(u)
    for b in range(B):
        for t in range(int(Tb[b])):
            out[b, t] = u[b, min(t + 1, int(Tb[b]) - 1)]
    return out


def receding_horizon(P, x0, cost, lo, hi, steps, T=None, K=5, tol=0.0, warm=True, plant=None, affine=None):
    """Closed-loop MPC (Sec. III-A; the outer loops of Alg. 1 and Alg. 2): at each step solve the
    horizon problem from the current state, apply the first control of the
    solution to the plant, and repeat from the state reached.

    cost: (Q, p) for a time-invariant cost, or a callable (step, x) -> (Q, p).
    warm: start each solve after the first from the shifted previous solution
    (shift_warm_start); otherwise every solve starts from hover thrust.
    plant: callable (x [B,13], u [B,4]) -> x_next; default one RK4 step of
    the quadrotor model per instance.  An instance with T_b = 0 keeps its
    state and applies zero controls.
    Returns dict(x [steps+1,B,13], u [steps,B,4], iters [steps,B],
    status [steps,B], u_star [steps,B,T,4], x_star [steps,B,T,13])."""
    x = _d(x0).copy()
    B = x.shape[0]
    Tb = None if T is None else np.asarray(T, np.int32)
    xs, us, its, sts, ustar, xstar = [x.copy()], [], [], [], [], []
    u_init = None
    for k in range(steps):
        Qk, pk = cost(k, x) if callable(cost) else cost
        out = forward(P, x, Qk, pk, lo, hi, T=Tb, K=K, tol=tol, affine=affine, u_init=u_init)
        u0 = out["u"][:, 0].copy()
        live = np.ones(B, bool) if Tb is None else Tb > 0
        if plant is not None:
            xn = plant(x, u0)
        else:
            xn = np.stack([rk4(P, x[b], u0[b]) for b in range(B)])
        x = np.where(live[:, None], xn, x)
        u_init = shift_warm_start(out["u"], Tb) if warm else None
        xs.append(x.copy())
        us.append(u0)
        its.append(out["iters"].copy())
        sts.append(out["status"].copy())
        ustar.append(out["u"].copy())
        xstar.append(out["x"].copy())
    return dict(x=np.array(xs), u=np.array(us), iters=np.array(its), status=np.array(sts), u_star=np.array(ustar),
                x_star=np.array(xstar))
