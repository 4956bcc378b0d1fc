"""The algebra of the time-parallel Riccati, written out in numpy and checked
against the FP64 oracle's own LQ solutions (CPU only).

The GPU form builds one element per stage (the stage's conditional value
function with the cross term and the clamped controls removed), combines them
with an associative operator in a suffix scan, and reads V_{t+1}, v_{t+1} off
the suffix products.  On an affine LQ problem the oracle's iLQR lands on the
optimum in one iteration, so the controls that the scanned value functions
produce (gains from V_{t+1}, v_{t+1}, rolled out from the start state) must be
the oracle's solution, with bounds whose active set the oracle reports held
fixed."""
import numpy as np
import pytest

import oracle as orc

NX, NU = 13, 4


def elements(A, Bm, C, g, pattern, kc):
    """One element (A, b, C, eta, J) per stage; pattern[t][a] True = clamped
    at the deviation kc[t][a]; the last stage's element is terminal."""
    T = len(C)
    out = []
    for t in range(T):
        f = [a for a in range(NU) if not pattern[t][a]]
        c = [a for a in range(NU) if pattern[t][a]]
        Cxx, Cxu, Cuu = C[t][:NX, :NX], C[t][:NX, NX:], C[t][NX:, NX:]
        gx, gu = g[t][:NX], g[t][NX:]
        kcv = np.array([kc[t][a] for a in c])
        Cxf, Cxc = Cxu[:, f], Cxu[:, c]
        r = Cuu[np.ix_(f, c)] @ kcv + gu[f]
        iR = np.linalg.inv(Cuu[np.ix_(f, f)]) if f else np.zeros((0, 0))
        J = Cxx - Cxf @ iR @ Cxf.T
        q = gx + Cxc @ kcv - Cxf @ iR @ r
        if t == T - 1:
            out.append((np.zeros((NX, NX)), np.zeros(NX), np.zeros((NX, NX)), -q, J))
            continue
        Bf, Bc = Bm[t][:, f], Bm[t][:, c]
        out.append((A[t] - Bf @ iR @ Cxf.T, Bc @ kcv - Bf @ iR @ r, Bf @ iR @ Bf.T, -q, J))
    return out


def combine(ei, ej):
    Ai, bi, Ci, ei_, Ji = ei
    Aj, bj, Cj, ej_, Jj = ej
    Mi = np.linalg.inv(np.eye(NX) + Ci @ Jj)
    return (Aj @ Mi @ Ai, Aj @ Mi @ (bi + Ci @ ej_) + bj, Aj @ Mi @ Ci @ Aj.T + Cj,
            Ai.T @ Mi.T @ (ej_ - Jj @ bi) + ei_, Ai.T @ Mi.T @ Jj @ Ai + Ji)


def suffix_scan(E):
    S, step = list(E), 1
    while step < len(S):
        S = [combine(S[t], S[t + step]) if t + step < len(S) else S[t] for t in range(len(S))]
        step *= 2
    return S


def rollout_from_scan(A, Bm, C, g, pattern, kc, S):
    """Gains of every stage from V_{t+1} = J, v_{t+1} = -eta of suffix t+1,
    then the controls from dx_0 = 0."""
    T = len(C)
    x, us = np.zeros(NX), []
    for t in range(T):
        F = np.hstack([A[t], Bm[t]]) if t + 1 < T else np.zeros((NX, NX + NU))
        V, v = (S[t + 1][4], -S[t + 1][3]) if t + 1 < T else (np.zeros((NX, NX)), np.zeros(NX))
        Q, q = C[t] + F.T @ V @ F, g[t] + F.T @ v
        f = [a for a in range(NU) if not pattern[t][a]]
        c = [a for a in range(NU) if pattern[t][a]]
        u = np.zeros(NU)
        u[c] = [kc[t][a] for a in c]
        if f:
            u[f] = -np.linalg.solve(Q[NX:, NX:][np.ix_(f, f)], q[NX:][f] + Q[NX:, NX:][np.ix_(f, c)] @ u[c]
                                    + Q[NX:, :NX][f] @ x)
        us.append(u)
        if t + 1 < T:
            x = A[t] @ x + Bm[t] @ u
    return np.array(us)


def random_lq(rng, T, dense):
    A = [np.eye(NX) + 0.15 * rng.normal(size=(NX, NX)) for _ in range(T)]
    Bm = [0.3 * rng.normal(size=(NX, NU)) for _ in range(T)]
    if dense:
        C = []
        for _ in range(T):
            G = rng.normal(size=(34, NX + NU))
            C.append(G.T @ G / 34 + 0.05 * np.eye(NX + NU))
    else:
        C = [np.diag(np.r_[10 ** rng.uniform(-1, 1, NX), rng.uniform(0.05, 0.5, NU)]) for _ in range(T)]
    g = [rng.normal(size=NX + NU) for _ in range(T)]
    return A, Bm, C, g


def oracle_lq(P, A, Bm, C, g, lo, hi):
    T = len(C)
    Aff = np.array(A)[None]
    Bff = np.array(Bm)[None]
    r = np.zeros((1, T, NX))
    iu = np.triu_indices(NX + NU)
    Q = np.array([Ct[iu] for Ct in C])[None]
    p = np.array(g)[None]
    return orc.forward(P, np.zeros((1, NX)), Q, p, lo[None], hi[None], K=60, tol=1e-15, affine=(Aff, Bff, r))


@pytest.mark.parametrize("dense", [False, True])
def test_scan_reproduces_the_oracle_lq_solution_without_bounds(P, dense):
    rng = np.random.default_rng(11 + dense)
    T = 9
    A, Bm, C, g = random_lq(rng, T, dense)
    free = [[False] * NU for _ in range(T)]
    S = suffix_scan(elements(A, Bm, C, g, free, [[0.0] * NU] * T))
    u = rollout_from_scan(A, Bm, C, g, free, [[0.0] * NU] * T, S)
    o = oracle_lq(P, A, Bm, C, g, np.full(NU, -1e30), np.full(NU, 1e30))
    assert o["status"][0] & orc.ST_CONVERGED
    assert np.abs(u - o["u"][0]).max() <= 1e-9 * max(1.0, np.abs(u).max())


@pytest.mark.parametrize("dense", [False, True])
def test_scan_with_the_oracle_active_set(P, dense):
    rng = np.random.default_rng(21 + dense)
    T = 8
    A, Bm, C, g = random_lq(rng, T, dense)
    g = [gt * 4.0 for gt in g]  # push some controls onto the bounds
    lo, hi = np.full(NU, -0.6), np.full(NU, 0.6)
    o = oracle_lq(P, A, Bm, C, g, lo, hi)
    assert o["status"][0] & orc.ST_CONVERGED
    uo = o["u"][0]
    pattern = [[bool(uo[t, a] == lo[a] or uo[t, a] == hi[a]) for a in range(NU)] for t in range(T)]
    assert 0 < sum(map(sum, pattern)) < T * NU
    kc = [[float(uo[t, a]) for a in range(NU)] for t in range(T)]
    S = suffix_scan(elements(A, Bm, C, g, pattern, kc))
    u = rollout_from_scan(A, Bm, C, g, pattern, kc, S)
    assert np.abs(u - uo).max() <= 1e-9 * max(1.0, np.abs(u).max())


def test_combination_is_associative(P):
    rng = np.random.default_rng(31)
    A, Bm, C, g = random_lq(rng, 4, False)
    free = [[False] * NU] * 4
    E = elements(A, Bm, C, g, free, [[0.0] * NU] * 4)
    left = combine(combine(E[0], E[1]), E[2])
    right = combine(E[0], combine(E[1], E[2]))
    for a, b in zip(left, right):
        assert np.allclose(a, b, rtol=1e-10, atol=1e-10 * max(1.0, np.abs(a).max()))
