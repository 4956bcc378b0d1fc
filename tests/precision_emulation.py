"""CPU emulation of the forward solve's arithmetic with the precision of each
step chosen separately.  It exists to decide, and to keep checkable, which
steps of the GPU forward need FP64 to meet the 1e-4 bar on u*.

The emulation follows the order of the kernel's stage algebra (Sec. IV:
rollout and linearisation, Riccati backward pass with input bounds, forward
pass with line search) for one instance at a time:

  linearisation   [A | B] = exact derivative of the RK4 map (chain rule
                  through the four stages), from the nominal (x, u)
  cost gradient   g = C z + c
  Q-function      Y = V F,  Q = C + F^T Y,  q = g + F^T v       (F = [A | B])
  control block   H = Q_uu factored as L D L^T with clamped rows/columns
                  replaced by the identity; k from the replayed clamp pattern,
                  K[f, :] = -H_ff^-1 Q_ux,f, K[clamped, :] = 0
  value update    V = Q_xx + Q_ux^T K,  v = Q_x + Q_ux^T k, V kept exactly
                  symmetric (upper triangle formed, mirrored)
  line search     u = clamp(u_bar + alpha k + K (x - x_bar)), x' = RK4(x, u)

with the discrete decisions (line-search index per iteration, clamp pattern
per stage, iteration count) replayed from a given run, so that a difference
from the FP64 oracle with the same decisions is arithmetic alone.

Precision switches (numpy dtypes), one per step:
  lin     the linearisation (RK4 and its chain rule)
  roll    the line-search rollout (control law, RK4) and the initial rollout
  traj    the nominal trajectory as kept between iterations
  acc     g, Y, Q and q
  vupd    the V, v update
  fact    the control-block factorisation and solves
  vstore  V, v as carried from one stage to the next
  gains   K, k as stored for the line search

KERNEL is the GPU forward's choice; FP64 everywhere reproduces the oracle.
Test infrastructure only; imports nothing from the HIP package.
"""
import numpy as np

NX, NU, NZ = 13, 4, 17
f32, f64 = np.float32, np.float64

KERNEL = dict(lin=f32, roll=f32, traj=f32, acc=f64, vupd=f64, fact=f64, vstore=f64, gains=f32)
ALL64 = dict(lin=f64, roll=f64, traj=f64, acc=f64, vupd=f64, fact=f64, vstore=f64, gains=f64)


def variant(**kw):
    p = dict(KERNEL)
    p.update(kw)
    return p


# ---------------------------------------------------------------------------
# quadrotor model (X configuration, scalar-first quaternion, body rates)
# ---------------------------------------------------------------------------

class Model:
    def __init__(self, P, dt):
        t = dt
        self.t = t
        self.h = t(P["dt"])
        self.g = t(P["g"])
        self.m = t(P["mass"])
        self.a = t(P["arm"] / np.sqrt(2.0))
        self.kap = t(P["kappa"])
        J = [t(P["Jxx"]), t(P["Jyy"]), t(P["Jzz"])]
        self.J = J
        self.c = [t((P["Jzz"] - P["Jyy"]) / P["Jxx"]), t((P["Jxx"] - P["Jzz"]) / P["Jyy"]),
                  t((P["Jyy"] - P["Jxx"]) / P["Jzz"])]
        # input map of (thrust / m, torques / J) per rotor
        mx, my, mz = np.array([1, 1, -1, -1]), np.array([-1, 1, 1, -1]), np.array([1, -1, 1, -1])
        self.Gu = np.stack([np.ones(4) / P["mass"], P["arm"] / np.sqrt(2.0) * mx / P["Jxx"],
                            P["arm"] / np.sqrt(2.0) * my / P["Jyy"], P["kappa"] * mz / P["Jzz"]]).astype(t)

    def inputs(self, u):
        s = (u[0] + u[1] + u[2] + u[3]) / self.m
        tx = self.a * (u[0] + u[1] - u[2] - u[3]) / self.J[0]
        ty = self.a * (-u[0] + u[1] + u[2] - u[3]) / self.J[1]
        tz = self.kap * (u[0] - u[1] + u[2] - u[3]) / self.J[2]
        return s, tx, ty, tz

    def rhs(self, x, u):
        t = self.t
        s, tx, ty, tz = self.inputs(u)
        qw, qx, qy, qz, wx, wy, wz = x[3], x[4], x[5], x[6], x[10], x[11], x[12]
        half, two = t(0.5), t(2.0)
        o = np.empty(NX, t)
        o[0:3] = x[7:10]
        o[3] = half * (-qx * wx - qy * wy - qz * wz)
        o[4] = half * (qw * wx + qy * wz - qz * wy)
        o[5] = half * (qw * wy - qx * wz + qz * wx)
        o[6] = half * (qw * wz + qx * wy - qy * wx)
        o[7] = s * (two * (qx * qz + qw * qy))
        o[8] = s * (two * (qy * qz - qw * qx))
        o[9] = s * (t(1.0) - two * (qx * qx + qy * qy)) - self.g
        o[10] = tx - self.c[0] * wy * wz
        o[11] = ty - self.c[1] * wz * wx
        o[12] = tz - self.c[2] * wx * wy
        return o

    def jac(self, x, u):
        """[F_x | F_u] of the right-hand side, 13 x 17."""
        t = self.t
        s = (u[0] + u[1] + u[2] + u[3]) / self.m
        qw, qx, qy, qz, wx, wy, wz = x[3], x[4], x[5], x[6], x[10], x[11], x[12]
        M = np.zeros((NX, NZ), t)
        M[0, 7] = M[1, 8] = M[2, 9] = 1
        h = t(0.5)
        Om = np.array([[0, -wx, -wy, -wz], [wx, 0, wz, -wy], [wy, -wz, 0, wx], [wz, wy, -wx, 0]], t)
        Xi = np.array([[-qx, -qy, -qz], [qw, -qz, qy], [qz, qw, -qx], [-qy, qx, qw]], t)
        M[3:7, 3:7] = h * Om
        M[3:7, 10:13] = h * Xi
        s2, s4 = s * t(2), s * t(4)
        M[7, 3:7] = [s2 * qy, s2 * qz, s2 * qw, s2 * qx]
        M[8, 3:7] = [-s2 * qx, -s2 * qw, s2 * qz, s2 * qy]
        M[9, 4:6] = [-s4 * qx, -s4 * qy]
        M[10, 11], M[10, 12] = -self.c[0] * wz, -self.c[0] * wy
        M[11, 10], M[11, 12] = -self.c[1] * wz, -self.c[1] * wx
        M[12, 10], M[12, 11] = -self.c[2] * wy, -self.c[2] * wx
        b3 = np.array([t(2) * (qx * qz + qw * qy), t(2) * (qy * qz - qw * qx), t(1) - t(2) * (qx * qx + qy * qy)], t)
        M[7:10, 13:17] = b3[:, None] * self.Gu[0][None, :]
        M[10:13, 13:17] = self.Gu[1:4]
        return M

    def rk4(self, x, u):
        h, h2, h6 = self.h, self.h * self.t(0.5), self.h / self.t(6)
        k1 = self.rhs(x, u)
        k2 = self.rhs(x + h2 * k1, u)
        k3 = self.rhs(x + h2 * k2, u)
        k4 = self.rhs(x + h * k3, u)
        return x + h6 * (k1 + self.t(2) * k2 + self.t(2) * k3 + k4)

    def rk4_jac(self, x, u):
        """[A | B] = d RK4(x, u) / d(x, u) by the chain rule through the stages."""
        t = self.t
        h, h2, h6 = self.h, self.h * t(0.5), self.h / t(6)
        I0 = np.zeros((NX, NZ), t)
        I0[:, :NX] = np.eye(NX, dtype=t)
        k1 = self.rhs(x, u)
        M1 = self.jac(x, u)
        x2 = x + h2 * k1
        J2 = self.jac(x2, u)
        M2 = J2[:, :NX] @ (I0 + h2 * M1)
        M2[:, NX:] += J2[:, NX:]
        k2 = self.rhs(x2, u)
        x3 = x + h2 * k2
        J3 = self.jac(x3, u)
        M3 = J3[:, :NX] @ (I0 + h2 * M2)
        M3[:, NX:] += J3[:, NX:]
        k3 = self.rhs(x3, u)
        x4 = x + h * k3
        J4 = self.jac(x4, u)
        M4 = J4[:, :NX] @ (I0 + h * M3)
        M4[:, NX:] += J4[:, NX:]
        return I0 + h6 * (M1 + t(2) * M2 + t(2) * M3 + M4)


# ---------------------------------------------------------------------------
# control block: L D L^T of the masked 4 x 4 block (clamped rows and columns
# replaced by the identity), no pivoting
# ---------------------------------------------------------------------------

def ldl_solve(H, fr, R, stats=None):
    """Solve Ht X = R, Ht = H with clamped rows/columns (fr == 0) replaced by
    the identity, by L D L^T in H's dtype.  R: [4] or [4, n].  stats: dict
    whose "min_pivot" is lowered to the smallest pivot D_j of a free row."""
    t = H.dtype.type
    Ht = H * np.outer(fr, fr)
    Ht[np.diag_indices(NU)] = np.where(fr != 0, np.diag(H), t(1))
    L = np.eye(NU, dtype=t)
    D = np.zeros(NU, t)
    for j in range(NU):
        D[j] = Ht[j, j] - np.sum(L[j, :j] ** 2 * D[:j])
        for i in range(j + 1, NU):
            L[i, j] = (Ht[i, j] - np.sum(L[i, :j] * L[j, :j] * D[:j])) / D[j]
    if stats is not None and np.any(fr != 0):
        stats["min_pivot"] = min(stats.get("min_pivot", np.inf), float(np.min(D[fr != 0])))
    Y = np.array(R, t)
    for i in range(NU):
        Y[i] = Y[i] - L[i, :i] @ Y[:i]
    Y = Y / (D if Y.ndim == 1 else D[:, None])
    for i in range(NU - 1, -1, -1):
        Y[i] = Y[i] - L[i + 1:, i] @ Y[i + 1:]
    return Y


def full_cost(q):
    if q.shape[-1] == NZ:
        return np.diag(q)
    C = np.zeros((NZ, NZ), q.dtype)
    iu = np.triu_indices(NZ)
    C[iu] = q
    return C + np.triu(C, 1).T


# ---------------------------------------------------------------------------
# the forward solve, decisions replayed
# ---------------------------------------------------------------------------

def forward_one(P, x0, Q, p, lo, hi, T, iters, alpha, pattern, alphas, prec, stats=None):
    """One instance.  Q [T_max, 17|153], p [T_max, 17] (float32 values),
    iters / alpha [K] / pattern [K, T_max] as in the decision log.  Returns
    u [T_max, 4], x [T_max, 13] as float64 (zero past T).  stats (a dict, or
    None) receives the smallest control-block pivot met ("min_pivot")."""
    ln, ro, tj, ac, vu, fa, vs, gn = (prec[k] for k in ("lin", "roll", "traj", "acc", "vupd", "fact", "vstore",
                                                          "gains"))
    Tm = p.shape[0]
    u_out, x_out = np.zeros((Tm, NU)), np.zeros((Tm, NX))
    if T <= 0:
        return u_out, x_out
    ml, mr = Model(P, ln), Model(P, ro)
    lo_r, hi_r = lo.astype(ro), hi.astype(ro)
    C = [full_cost(Q[t].astype(ac)) for t in range(T)]
    c = [p[t].astype(ac) for t in range(T)]
    # U^0: hover thrust m g / 4 (formed in the rollout's precision), clamped
    hover = ro(ro(P["mass"]) * ro(P["g"]) / ro(4))
    U = np.clip(np.full((T, NU), hover, ro), lo_r, hi_r).astype(ro)
    X = np.zeros((T, NX), ro)
    X[0] = x0.astype(ro)
    for t in range(T - 1):
        X[t + 1] = mr.rk4(X[t], U[t])
    X, U = X.astype(tj), U.astype(tj)
    for k in range(int(iters)):
        F = [ml.rk4_jac(X[t].astype(ln), U[t].astype(ln)) for t in range(T - 1)]
        V = np.zeros((NX, NX), vs)
        v = np.zeros(NX, vs)
        Kst = np.zeros((T, NU, NX), gn)
        kst = np.zeros((T, NU), gn)
        for t in range(T - 1, -1, -1):
            z = np.concatenate([X[t], U[t]]).astype(ac)
            g = C[t] @ z + c[t]
            if t + 1 < T:
                Fa = F[t].astype(ac)
                Y = V.astype(ac) @ Fa
                Qm = C[t] + Fa.T @ Y
                q = g + Fa.T @ v.astype(ac)
            else:
                Qm, q = C[t].copy(), g
            code = int(pattern[k, t])
            pat = np.array([(code >> (2 * i)) & 3 for i in range(NU)])
            fr = (pat == 0).astype(fa)
            H = Qm[NX:, NX:].astype(fa)
            qu = q[NX:].astype(fa)
            Qux = Qm[NX:, :NX].astype(fa)
            a = (lo.astype(f64) - U[t].astype(f64)).astype(fa)
            b = (hi.astype(f64) - U[t].astype(f64)).astype(fa)
            kc = np.where(pat == 1, a, np.where(pat == 2, b, 0)).astype(fa)
            # free part: H_ff k_f = -(q_f + H_fc k_c)
            rhs = -(qu + H @ kc) * fr
            kk = ldl_solve(H, fr, rhs, stats) * fr + kc
            kk = np.clip(kk, a, b)
            KK = -ldl_solve(H, fr, Qux * fr[:, None]) * fr[:, None]
            Qx = q[:NX].astype(vu)
            Vn = Qm[:NX, :NX].astype(vu) + Qux.astype(vu).T @ KK.astype(vu)
            vn = Qx + Qux.astype(vu).T @ kk.astype(vu)
            Vn = np.triu(Vn) + np.triu(Vn, 1).T
            V, v = Vn.astype(vs), vn.astype(vs)
            Kst[t], kst[t] = KK.astype(gn), kk.astype(gn)
        ai = int(alpha[k])
        if ai == 255:
            continue
        al = ro(alphas[ai])
        Xn, Un = np.zeros(X.shape, ro), np.zeros(U.shape, ro)
        x = x0.astype(ro)
        Xr, Ur = X.astype(ro), U.astype(ro)
        for t in range(T):
            ur = Ur[t] + al * kst[t].astype(ro) + Kst[t].astype(ro) @ (x - Xr[t])
            ur = np.clip(ur, lo_r, hi_r).astype(ro)
            Xn[t], Un[t] = x, ur
            if t + 1 < T:
                x = mr.rk4(x, ur)
        X, U = Xn.astype(tj), Un.astype(tj)
    u_out[:T], x_out[:T] = U, X
    return u_out, x_out


def forward(P, d, dec, prec, alphas, idx=None, stats=None):
    """Batch wrapper: d a workload dict (float32 arrays), dec = (iters [B],
    alpha [B, K], pattern [B, K, T_max]) for the instances idx (all when None).
    Returns u [n, T_max, 4], x [n, T_max, 13]; stats (a list, or None) gets one
    dict per instance (see forward_one)."""
    idx = range(d["B"]) if idx is None else idx
    us, xs = [], []
    for j, b in enumerate(idx):
        st = {} if stats is not None else None
        u, x = forward_one(P, d["x0"][b], d["Q"][b], d["p"][b], d["lo"][b], d["hi"][b], int(d["T"][b]),
                           dec[0][j], dec[1][j], dec[2][j], alphas, prec, st)
        if stats is not None:
            stats.append(st)
        us.append(u)
        xs.append(x)
    return np.array(us), np.array(xs)
