"""Pins of the oracle's iLQR (Alg. 2 inner loop; Sec. IV three-stage loop) and
of its two backwards (Sec. IV after eq. (3): implicit KKT differentiation).

On affine dynamics the OCP of eq. (3) is a convex QP, so:
  * with no active bounds one iLQR iteration lands on the optimum, which is
    the solution of the equality-constrained KKT system (numpy solve);
  * with bounds, the optimum is found by brute force over every active set of
    the condensed QP in U (3^{4T} patterns, T <= 3);
  * the Riccati-adjoint backward must equal the dense KKT backward.
"""
import itertools
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def affine_problem(rng, B, T, dense=False, bound=None, pu=1.0):
    A = np.eye(13)[None, None] + 0.15 * rng.normal(size=(B, T, 13, 13))
    Bm = 0.3 * rng.normal(size=(B, T, 13, 4))
    r = 0.1 * rng.normal(size=(B, T, 13))
    x0 = rng.normal(size=(B, 13))
    if dense:
        G = rng.normal(size=(B, T, 34, 17))
        S = np.einsum("btki,btkj->btij", G, G) / 34 + 0.05 * np.eye(17)
        iu = np.triu_indices(17)
        Q = S[..., iu[0], iu[1]]
    else:
        Q = np.concatenate([10 ** rng.uniform(-1, 1, size=(B, T, 13)), rng.uniform(0.05, 0.5, size=(B, T, 4))], -1)
    p = rng.normal(size=(B, T, 17))
    p[..., 13:] *= pu
    if bound is None:
        lo, hi = np.full((B, 4), -1e30), np.full((B, 4), 1e30)
    else:
        lo, hi = np.full((B, 4), -bound), np.full((B, 4), bound)
    return dict(affine=(A, Bm, r), x0=x0, Q=Q, p=p, lo=lo, hi=hi)


def full_cost(Q):
    if Q.shape[-1] == 17:
        return np.diag(Q)
    C = np.zeros((17, 17))
    iu = np.triu_indices(17)
    C[iu] = Q
    return C + np.triu(C, 1).T


def condensed(pr, b, T):
    A, Bm, r = (a[b] for a in pr["affine"])
    x0 = pr["x0"][b]

    def traj(U):
        x, zs = x0, []
        for t in range(T):
            u = U[4 * t:4 * t + 4]
            zs.append(np.concatenate([x, u]))
            if t < T - 1:
                x = A[t] @ x + Bm[t] @ u + r[t]
        return np.concatenate(zs)

    m0 = traj(np.zeros(4 * T))
    M = np.stack([traj(np.eye(4 * T)[j]) - m0 for j in range(4 * T)], axis=1)
    H = np.zeros((17 * T, 17 * T))
    for t in range(T):
        H[17 * t:17 * t + 17, 17 * t:17 * t + 17] = full_cost(pr["Q"][b, t])
    c = pr["p"][b].reshape(-1)
    return M.T @ H @ M, M.T @ (H @ m0 + c), M, m0


def brute_force_boxqp(Hu, hu, lo, hi):
    """Unique minimiser of a strictly convex box-QP by checking every active set."""
    n = len(hu)
    best = None
    pats = np.array(list(itertools.product((0, 1, 2), repeat=n)))
    for s in range(0, len(pats), 20000):
        P = pats[s:s + 20000]
        m = len(P)
        Ht = np.broadcast_to(Hu, (m, n, n)).copy()
        rhs = np.broadcast_to(-hu, (m, n)).copy()
        clamped = P != 0
        bnd = np.where(P == 1, lo, hi)
        ii = np.arange(n)
        for i in range(n):
            sel = clamped[:, i]
            Ht[sel, i, :] = 0.0
            Ht[sel, i, i] = 1.0
            rhs[sel, i] = bnd[sel, i]
        U = np.linalg.solve(Ht, rhs[..., None])[..., 0]
        g = U @ Hu.T + hu
        tol = 1e-9 * (1 + np.abs(hu).max())
        ok = np.all(np.where(P == 0, (U >= lo - 1e-9) & (U <= hi + 1e-9), True), axis=1)
        ok &= np.all(np.where(P == 1, g >= -tol, True), axis=1)
        ok &= np.all(np.where(P == 2, g <= tol, True), axis=1)
        idx = np.nonzero(ok)[0]
        if len(idx):
            best = U[idx[0]]
            break
    assert best is not None
    return best


@pytest.mark.parametrize("dense", [False, True])
def test_unconstrained_lqr_one_iteration_is_kkt_solution(orc, P, dense):
    rng = np.random.default_rng(11 + dense)
    B, T = 3, 6
    pr = affine_problem(rng, B, T, dense=dense)
    f = orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], K=1, affine=pr["affine"])
    assert (f["alpha"][:, 0] == 0).all()  # the full Newton step wins
    for b in range(B):
        A, Bm, r = (a[b] for a in pr["affine"])
        nz, nc = 17 * T, 13 * T
        M = np.zeros((nz + nc, nz + nc))
        rhs = np.zeros(nz + nc)
        for t in range(T):
            M[17 * t:17 * t + 17, 17 * t:17 * t + 17] = full_cost(pr["Q"][b, t])
            rhs[17 * t:17 * t + 17] = -pr["p"][b, t]
        G = np.zeros((nc, nz))
        h = np.zeros(nc)
        G[0:13, 0:13] = np.eye(13)
        h[0:13] = pr["x0"][b]
        for t in range(T - 1):
            rw = 13 * (t + 1)
            G[rw:rw + 13, 17 * (t + 1):17 * (t + 1) + 13] = np.eye(13)
            G[rw:rw + 13, 17 * t:17 * t + 13] = -A[t]
            G[rw:rw + 13, 17 * t + 13:17 * t + 17] = -Bm[t]
            h[rw:rw + 13] = r[t]
        M[nz:, :nz] = G
        M[:nz, nz:] = G.T
        rhs[nz:] = h
        z = np.linalg.solve(M, rhs)[:nz].reshape(T, 17)
        assert np.abs(f["u"][b] - z[:, 13:]).max() <= 1e-10 * max(1, np.abs(z).max())
        assert np.abs(f["x"][b] - z[:, :13]).max() <= 1e-10 * max(1, np.abs(z).max())


@pytest.mark.parametrize("T,seed", [(1, 0), (2, 1), (2, 2), (2, 3), (3, 4)])
def test_box_lq_matches_brute_force(orc, P, T, seed):
    rng = np.random.default_rng(100 + seed)
    pr = affine_problem(rng, 1, T, bound=0.6, pu=3.0)
    f = orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], K=300, tol=1e-14, affine=pr["affine"])
    assert f["status"][0] & orc.ST_CONVERGED
    Hu, hu, M, m0 = condensed(pr, 0, T)
    U = brute_force_boxqp(Hu, hu, pr["lo"][0, 0], pr["hi"][0, 0])
    assert np.abs(f["u"][0].reshape(-1) - U).max() <= 1e-9
    # some bound must be active for the case to be meaningful
    assert np.any(np.isclose(np.abs(U), 0.6))


@pytest.mark.parametrize("dense", [False, True])
def test_riccati_adjoint_equals_dense_kkt(orc, P, dense):
    rng = np.random.default_rng(21 + dense)
    B, T = 4, 8
    pr = affine_problem(rng, B, T, dense=dense, bound=0.8)
    f = orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], K=20, affine=pr["affine"])
    gu = rng.normal(size=(B, T, 4))
    gx = rng.normal(size=(B, T, 13))
    args = (P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], f["u"], f["x"], gu, gx)
    r0 = orc.backward(*args, method=0, affine=pr["affine"])
    r1 = orc.backward(*args, method=1, affine=pr["affine"])
    for k in ("dQ", "dp", "dx0"):
        assert np.abs(r0[k] - r1[k]).max() <= 1e-10 * max(1, np.abs(r1[k]).max()), k


def test_riccati_adjoint_equals_dense_kkt_quadrotor(orc, P):
    import workloads as W
    d = W.make(0)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    args = (P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"], d["grad_u"])
    r0 = orc.backward(*args, method=0)
    r1 = orc.backward(*args, method=1)
    for k in ("dQ", "dp", "dx0"):
        assert np.abs(r0[k] - r1[k]).max() <= 1e-10 * max(1, np.abs(r1[k]).max()), k


def kkt_optimum(pr, b, T):
    """The unconstrained optimum of instance b over its first T stages (dense
    equality-constrained KKT solve, numpy) as z [T, 17]."""
    A, Bm, r = (a[b] for a in pr["affine"])
    nz, nc = 17 * T, 13 * T
    M = np.zeros((nz + nc, nz + nc))
    rhs = np.zeros(nz + nc)
    for t in range(T):
        M[17 * t:17 * t + 17, 17 * t:17 * t + 17] = full_cost(pr["Q"][b, t])
        rhs[17 * t:17 * t + 17] = -pr["p"][b, t]
    G = np.zeros((nc, nz))
    h = np.zeros(nc)
    G[0:13, 0:13] = np.eye(13)
    h[0:13] = pr["x0"][b]
    for t in range(T - 1):
        rw = 13 * (t + 1)
        G[rw:rw + 13, 17 * (t + 1):17 * (t + 1) + 13] = np.eye(13)
        G[rw:rw + 13, 17 * t:17 * t + 13] = -A[t]
        G[rw:rw + 13, 17 * t + 13:17 * t + 17] = -Bm[t]
        h[rw:rw + 13] = r[t]
    M[nz:, :nz] = G
    M[:nz, nz:] = G.T
    rhs[nz:] = h
    return np.linalg.solve(M, rhs)[:nz].reshape(T, 17)


def objective(pr, b, z):
    """Eq. (3)'s objective sum_t 1/2 z_t^T C_t z_t + c_t^T z_t over the rows of z."""
    return sum(0.5 * z[t] @ full_cost(pr["Q"][b, t]) @ z[t] + pr["p"][b, t] @ z[t] for t in range(len(z)))


@pytest.mark.parametrize("dense", [False, True])
def test_line_search_costs_follow_the_newton_parabola(orc, P, dense):
    """Line search (Sec. IV "Forward pass with line-search") on an unbounded
    affine problem, one iteration from a random U^0.  The backward pass then
    gives the exact Newton step dz to the optimum, and the candidate with step
    length alpha is the trajectory z0 + alpha dz (the feedback term follows
    the state deviation, which is alpha dx by linearity).  Since the optimum
    makes the derivative of J(z0 + alpha dz) vanish at alpha = 1, the cost of
    the candidate is J0 + (J1 - J0)(2 alpha - alpha^2), with J0 the cost of
    U^0's rollout and J1 the optimal cost, both evaluated here in numpy.
    Pins the oracle's step lengths (against the paper's list), the 1/2 and
    the range of stages of its cost.  Ragged horizons with non-zero cost
    data past T_b: those stages must not count."""
    alphas = np.array(GOLD["line_search_alphas"])
    rng = np.random.default_rng(31 + dense)
    B, Tm = 3, 7
    pr = affine_problem(rng, B, Tm, dense=dense)
    T = np.array([7, 5, 1], np.int32)
    u0 = rng.normal(size=(B, Tm, 4))
    f = orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], T, K=1, affine=pr["affine"], u_init=u0)
    f0 = orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], T, K=0, affine=pr["affine"], u_init=u0)
    for b in range(B):
        Tb = int(T[b])
        A, Bm, r = (a[b] for a in pr["affine"])
        x, z0 = pr["x0"][b], []
        for t in range(Tb):
            z0.append(np.concatenate([x, u0[b, t]]))
            x = A[t] @ x + Bm[t] @ u0[b, t] + r[t]
        J0 = objective(pr, b, np.array(z0))
        J1 = objective(pr, b, kkt_optimum(pr, b, Tb))
        assert abs(f0["J"][b] - J0) <= 1e-10 * max(1.0, abs(J0))
        want = J0 + (J1 - J0) * (2 * alphas - alphas ** 2)
        scale = max(1.0, abs(J0), abs(J1))
        assert np.abs(f["cand_cost"][b, 0] - want).max() <= 1e-9 * scale, (b, f["cand_cost"][b, 0], want)
        assert f["alpha"][b, 0] == 0 and abs(f["J"][b] - J1) <= 1e-9 * scale


def test_replay_check_accepts_valid_and_flags_wrong_patterns(orc, P):
    """The replay of another solver's box-QP decisions scores each pattern
    against the oracle's own stage QP: the oracle's own patterns score 0, and
    a pattern with one coordinate wrongly put on a bound, or wrongly released
    from one, is flagged (the replay still clamps that step into the box, so
    the trajectory alone would not show it)."""
    import workloads as W
    d = W.make(0, pu_scale=0.01, seed=2000)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    rep = (f["iters"], f["alpha"], f["pattern"])
    g = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5, replay=rep)
    assert np.array_equal(g["u"], f["u"]) and g["replay_viol"].max() <= 1e-9
    codes = f["pattern"]
    planted = 0
    for kind in ("clamp_free", "free_clamped"):
        bad = codes.copy()
        hit = None
        for b, k, t in zip(*np.nonzero(np.ones(codes.shape, bool))):
            if k >= f["iters"][b] or t >= d["T"][b]:
                continue
            c = int(codes[b, k, t])
            for i in range(4):
                ci = (c >> (2 * i)) & 3
                if kind == "clamp_free" and ci == 0:
                    bad[b, k, t] = c | (1 << (2 * i))   # free -> lower bound
                    hit = (b, k, t)
                elif kind == "free_clamped" and ci != 0:
                    bad[b, k, t] = c & ~(3 << (2 * i))  # clamped -> free
                    hit = (b, k, t)
                if hit:
                    break
            if hit:
                break
        assert hit is not None, kind
        h = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5,
                        replay=(f["iters"], f["alpha"], bad))
        assert h["replay_viol"][hit] > 1e-3, (kind, h["replay_viol"][hit])
        planted += 1
    assert planted == 2


def test_line_search_takes_first_minimiser(orc, P):
    import workloads as W
    d = W.make(0)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    cc = f["cand_cost"]
    for b in range(d["B"]):
        for k in range(5):
            assert f["alpha"][b, k] == int(np.argmin(cc[b, k]))


def test_replay_of_own_decisions_is_identical(orc, P):
    import workloads as W
    d = W.make(0)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    g = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5,
                    replay=(f["iters"], f["alpha"], f["pattern"]))
    assert np.array_equal(f["u"], g["u"]) and np.array_equal(f["x"], g["x"])


def test_controls_stay_in_box_and_ragged_padding(orc, P):
    import workloads as W
    d = W.make(3, B=16, T=14)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=10, tol=1e-5)
    lo, hi = d["lo"][:, None, :], d["hi"][:, None, :]
    assert np.all(f["u"] >= lo) and np.all(f["u"] <= hi)
    pad = np.arange(14)[None, :] >= d["T"][:, None]
    assert np.all(f["u"][pad] == 0) and np.all(f["x"][pad] == 0)
    assert np.all((f["status"] & (orc.ST_CONVERGED | orc.ST_MAXITER)) != 0)


def test_degenerate_horizons(orc, P):
    import workloads as W
    d = W.make(0, B=3, T=4)
    T = np.array([0, 1, 4], np.int32)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], T, K=3)
    assert np.all(f["u"][0] == 0) and f["iters"][0] == 0
    # T = 1: u_0 minimises its own stage cost over the box: separable clamp
    q = d["Q"][1, 0, 13:].astype(np.float64)
    pu = d["p"][1, 0, 13:].astype(np.float64)
    assert np.allclose(f["u"][1, 0], np.clip(-pu / q, d["lo"][1], d["hi"][1]), rtol=0, atol=1e-12)
    r = orc.backward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"], d["grad_u"], T=T)
    assert np.all(r["dx0"][0] == 0) and np.all(r["dp"][0] == 0)
