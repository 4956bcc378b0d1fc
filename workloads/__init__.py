"""Seeded synthetic inputs for the batched differentiable-MPC workloads.

This module holds none of the method's arithmetic: it only draws random
numbers and shapes them into problem instances.  It is the one piece shared
by the HIP-path tests and the oracle tests.

The paper measures on a custom drone-racing environment with a reconstructed
track and on hover stabilisation (Sec. V); neither is available, so these
seeded generators stand in for them with the shapes and value ranges of the
five workloads:

  cfg 0  B=8,     T=10,  diagonal cost, x0 noise sigma 0.1 m  (oracle-sized)
  cfg 1  B=1024,  T=20,  diagonal cost, x0 position noise sigma 1 m, forward only
  cfg 2  B=4096,  T=20,  cost emitted by a random-init 2x256 tanh MLP
  cfg 3  B=8192,  T~U{10..50}, per-instance upper bound U[6,10], K<=10, tol 1e-5
  cfg 4  B=16384, T=50,  dense Wishart(34 dof) stage cost, condition <= 1e4

Arrays are float32 numpy, instance-major: x0 [B,13], Q [B,T,17|153],
p [B,T,17], lo/hi [B,4], T [B] int32, grad_u [B,T,4].
Draw order per config: x0 noise, Q, p, bounds, T, upstream gradient, MLP.
"""
import numpy as np

NX, NU, NZ, NPACK = 13, 4, 17, 153

# Quadrotor constants of the workloads (mass, inertia, arm, torque
# coefficient, RK4 step); g is this project's choice.
QUAD = dict(mass=0.75, Jxx=2.5e-3, Jyy=2.5e-3, Jzz=4.5e-3, arm=0.15, kappa=0.01, dt=0.05, g=9.81)

CONFIGS = {
    0: dict(B=8, T=10, cost="diag", pos_sigma=0.1, K=5, tol=0.0, seed=1000, grad="full"),
    1: dict(B=1024, T=20, cost="diag", pos_sigma=1.0, K=5, tol=0.0, seed=1001, grad=None),
    2: dict(B=4096, T=20, cost="mlp", pos_sigma=1.0, K=5, tol=0.0, seed=1002, grad="first"),
    3: dict(B=8192, T=50, cost="diag", pos_sigma=1.0, K=10, tol=1e-5, seed=1003, grad="full", ragged=(10, 50),
            hi_range=(6.0, 10.0)),
    4: dict(B=16384, T=50, cost="dense", pos_sigma=1.0, K=5, tol=0.0, seed=1004, grad="full", ckpt=10),
}


def quad_params_f32():
    """The constants rounded to float32 (what the FP32 kernels see), as Python
    floats so the FP64 oracle can be given exactly the same values."""
    return {k: float(np.float32(v)) for k, v in QUAD.items()}


def hover_state(B):
    x = np.zeros((B, NX), np.float64)
    x[:, 3] = 1.0
    return x


def _diag_cost(rng, B, T):
    q = 10.0 ** rng.uniform(-2.0, 2.0, size=(B, T, NX))
    Q = np.concatenate([q, np.full((B, T, NU), 1e-2)], axis=2)
    return Q


def _wishart_packed(rng, B, T, dof=34, cond_max=1e4, chunk=4096):
    """Packed-upper S = G^T G / dof, G ~ N(0,1)^{dof x 17}; if cond(S) exceeds
    cond_max add the ridge that brings it to exactly cond_max."""
    iu = np.triu_indices(NZ)
    out = np.empty((B * T, NPACK), np.float32)
    n = B * T
    for s in range(0, n, chunk):
        m = min(chunk, n - s)
        G = rng.standard_normal((m, dof, NZ))
        S = np.einsum("bki,bkj->bij", G, G) / dof
        w = np.linalg.eigvalsh(S)
        lmin, lmax = w[:, 0], w[:, -1]
        ridge = np.where(lmax > cond_max * lmin, (lmax - cond_max * lmin) / (cond_max - 1.0), 0.0)
        S = S + ridge[:, None, None] * np.eye(NZ)
        out[s:s + m] = S[:, iu[0], iu[1]].astype(np.float32)
    return out.reshape(B, T, NPACK)


class CostMLP:
    """Random-init cost map: concat(x0, gate) (25) -> 256 tanh -> 256 tanh ->
    T*(13+17).  Per stage the first 13 outputs give Q_x = 10^(4 sigmoid(h) - 2)
    in (1e-2, 1e2), R = 1e-2 I is fixed, and the last 17 are the linear term p
    (the sigmoid scaling mirrors the bounded output layer of the paper's actor,
    Sec. V "learning setup")."""

    def __init__(self, T, seed, device="cpu"):
        import torch
        g = torch.Generator().manual_seed(seed)
        self.T = T

        def lin(i, o):
            bound = 1.0 / np.sqrt(i)
            w = (torch.rand(o, i, generator=g, dtype=torch.float32) * 2 - 1) * bound
            b = (torch.rand(o, generator=g, dtype=torch.float32) * 2 - 1) * bound
            return w.to(device).requires_grad_(True), b.to(device).requires_grad_(True)

        self.params = [*lin(NX + 12, 256), *lin(256, 256), *lin(256, T * (NX + NZ))]

    def __call__(self, inp):
        import torch
        w1, b1, w2, b2, w3, b3 = self.params
        h = torch.tanh(inp @ w1.T + b1)
        h = torch.tanh(h @ w2.T + b2)
        o = (h @ w3.T + b3).reshape(inp.shape[0], self.T, NX + NZ)
        qx = 10.0 ** (4.0 * torch.sigmoid(o[..., :NX]) - 2.0)
        R = torch.full(qx.shape[:-1] + (NU,), 1e-2, dtype=qx.dtype, device=qx.device)
        Q = torch.cat([qx, R], dim=-1)
        p = o[..., NX:]
        return Q, p


def make(cfg_id, B=None, T=None, seed=None, pu_scale=1.0, r_scale=1.0):
    """Return the inputs of a workload as a dict of numpy arrays (float32) plus
    metadata.  B / T / seed override the configuration's values (smaller
    instances of the same distribution for tests).  pu_scale multiplies the
    control part of p (0.01 gives non-trivial free sets; default 1).  r_scale
    multiplies the control weight R of a diagonal cost (1e-6 gives R = 1e-8,
    the adversarial set whose Cholesky pivots fall below 1e-6)."""
    c = dict(CONFIGS[cfg_id])
    B = c["B"] if B is None else B
    Tm = c["T"] if T is None else T
    seed = c["seed"] if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    # x0: hover plus noise on position and velocity
    x0 = hover_state(B)
    x0[:, 0:3] += rng.normal(0.0, c["pos_sigma"], size=(B, 3))
    x0[:, 7:10] += rng.normal(0.0, 0.1, size=(B, 3))
    mlp = None
    gate = None
    if c["cost"] == "diag":
        Q = _diag_cost(rng, B, Tm)
        Q[..., NX:] *= r_scale
        p = rng.standard_normal((B, Tm, NZ))
    elif c["cost"] == "dense":
        Q = _wishart_packed(rng, B, Tm)
        p = rng.standard_normal((B, Tm, NZ))
    else:  # mlp: the gate vector is drawn here, the cost comes from the MLP below
        gate = rng.standard_normal((B, 12))
        Q = p = None
    if p is not None:
        p[..., NX:] *= pu_scale
    lo = np.zeros((B, NU))
    if "hi_range" in c:
        hi = np.repeat(rng.uniform(*c["hi_range"], size=(B, 1)), NU, axis=1)
    else:
        hi = np.full((B, NU), 8.5)
    if "ragged" in c:
        lo_T, hi_T = c["ragged"]
        hi_T = min(hi_T, Tm)
        lo_T = min(lo_T, hi_T)
        Tb = rng.integers(lo_T, hi_T + 1, size=B).astype(np.int32)
    else:
        Tb = np.full(B, Tm, np.int32)
    grad_u = np.zeros((B, Tm, NU))
    w = None
    if c["grad"] == "full":
        grad_u = rng.standard_normal((B, Tm, NU))
    elif c["grad"] == "first":
        w = rng.standard_normal((B, NU))
        grad_u[:, 0, :] = w
    grad_u[np.arange(Tm)[None, :] >= Tb[:, None]] = 0.0
    out = dict(x0=x0.astype(np.float32), lo=lo.astype(np.float32), hi=hi.astype(np.float32), T=Tb,
               grad_u=grad_u.astype(np.float32), K=c["K"], tol=c["tol"], T_max=Tm, B=B,
               cost_kind=1 if c["cost"] == "dense" else 0, ckpt=c.get("ckpt", 0), cfg=cfg_id)
    if c["cost"] == "mlp":
        import torch
        mlp = CostMLP(Tm, seed)
        inp = torch.from_numpy(np.concatenate([x0, gate], axis=1).astype(np.float32))
        with torch.no_grad():
            Qt, pt = mlp(inp)
        out["Q"] = Qt.numpy().astype(np.float32)
        out["p"] = pt.numpy().astype(np.float32)
        out["mlp"] = mlp
        out["mlp_input"] = inp.numpy()
        out["w"] = w.astype(np.float32)
    else:
        out["Q"] = Q.astype(np.float32)
        out["p"] = p.astype(np.float32)
    # padded stages beyond T_b carry zero cost
    pad = np.arange(Tm)[None, :] >= Tb[:, None]
    out["Q"][pad] = 0.0
    out["p"][pad] = 0.0
    return out


def make_hover_target(B, T, seed=1100, K=5):
    """Hover-to-target latency workload (the shapes of the paper's solver
    latency measurement, Sec. V-A / Table I): x0 is hover at the origin with
    N(0, 0.1) noise on position and velocity; each instance is asked to hover
    at a target position drawn uniformly in [-1, 1]^3 m.  The stage cost is
    1/2 (z - z_ref)^T C (z - z_ref) with C = diag(10 on position, 1 on the
    quaternion, 1 on velocity, 0.1 on body rates, 0.01 on the thrusts) and
    z_ref = (target, level attitude, zero velocity and rates, hover thrust),
    i.e. c = -C z_ref.  Controls boxed to [0, 8.5] N."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x0 = hover_state(B)
    x0[:, 0:3] += rng.normal(0.0, 0.1, size=(B, 3))
    x0[:, 7:10] += rng.normal(0.0, 0.1, size=(B, 3))
    target = rng.uniform(-1.0, 1.0, size=(B, 3))
    qd = np.array([10.0] * 3 + [1.0] * 4 + [1.0] * 3 + [0.1] * 3 + [0.01] * 4)
    hover_u = QUAD["mass"] * QUAD["g"] / 4.0
    zref = np.zeros((B, NZ))
    zref[:, 0:3] = target
    zref[:, 3] = 1.0
    zref[:, NX:] = hover_u
    Q = np.broadcast_to(qd, (B, T, NZ)).copy()
    p = -(Q * zref[:, None, :])
    lo = np.zeros((B, NU))
    hi = np.full((B, NU), 8.5)
    grad_u = rng.standard_normal((B, T, NU))
    return dict(x0=x0.astype(np.float32), Q=Q.astype(np.float32), p=p.astype(np.float32), lo=lo.astype(np.float32),
                hi=hi.astype(np.float32), T=np.full(B, T, np.int32), grad_u=grad_u.astype(np.float32), K=K, tol=0.0,
                T_max=T, B=B, cost_kind=0, ckpt=0, cfg="hover")
