"""Pins of the oracle's backward (Sec. IV after eq. (3): gradients of an
external loss w.r.t. (C_t, c_t, x_init) by implicit differentiation of the KKT
conditions at the solution, after Amos et al. 2018).

The backward differentiates the box-constrained LQ solution map Phi(theta) of
the model linearised at the solution, with the active set held fixed.  Within
one active-set region Phi is affine in (c, x_init), so central finite
differences of the oracle's own converged forward solve are exact up to
solver round-off; in C it is rational, so FD is O(h^2).
"""
import numpy as np
import pytest

from test_oracle_lqr import affine_problem


def solve(orc, P, pr, K=400, u_init=None):
    return orc.forward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], K=K, tol=1e-15, affine=pr["affine"],
                       u_init=u_init)


def loss(f, gu, gx):
    return np.sum(f["u"] * gu, axis=(1, 2)) + np.sum(f["x"] * gx, axis=(1, 2))


def mask(orc, f, pr):
    return orc.active_mask(f["u"], pr["lo"], pr["hi"])


def fd_check(orc, P, pr, base, gu, gx, key, index, h, rel_step=False):
    """Central FD of L along one input coordinate; returns (fd, ok) where ok is
    False when the active set changes inside [theta - h, theta + h]."""
    vals, masks = [], []
    for s in (+1, -1):
        q = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in pr.items()}
        arr = q[key]
        step = h * (abs(arr[index]) if rel_step else 1.0)
        arr[index] = arr[index] + s * step
        f = solve(orc, P, q, u_init=base["u"])
        vals.append(loss(f, gu, gx)[0])
        masks.append(mask(orc, f, pr))
    ok = np.array_equal(masks[0], masks[1]) and np.array_equal(masks[0], mask(orc, base, pr))
    return (vals[0] - vals[1]) / (2 * step), ok


@pytest.mark.parametrize("dense", [False, True])
def test_gradients_match_central_fd_affine(orc, P, dense):
    rng = np.random.default_rng(31 + dense)
    T = 5
    pr = affine_problem(rng, 1, T, dense=dense, bound=0.7, pu=2.0)
    base = solve(orc, P, pr)
    assert base["status"][0] & orc.ST_CONVERGED
    m = mask(orc, base, pr)
    assert 0 < bin(int(np.bitwise_or.reduce(m[0]))).count("1")  # some bound active
    gu = rng.normal(size=(1, T, 4))
    gx = rng.normal(size=(1, T, 13))
    g = orc.backward(P, pr["x0"], pr["Q"], pr["p"], pr["lo"], pr["hi"], base["u"], base["x"], gu, gx,
                     affine=pr["affine"])
    checked = 0
    for (t, i) in [(0, 0), (1, 5), (2, 13), (3, 15), (4, 16), (2, 9), (0, 14)]:
        fd, ok = fd_check(orc, P, pr, base, gu, gx, "p", (0, t, i), 1e-5)
        if ok:
            checked += 1
            assert abs(fd - g["dp"][0, t, i]) <= 1e-7 * max(1, abs(fd)), ("p", t, i)
    for i in (0, 3, 8, 12):
        fd, ok = fd_check(orc, P, pr, base, gu, gx, "x0", (0, i), 1e-5)
        if ok:
            checked += 1
            assert abs(fd - g["dx0"][0, i]) <= 1e-7 * max(1, abs(fd)), ("x0", i)
    for (t, j) in [(0, 0), (1, 3), (2, 14), (4, 16), (3, 40 if dense else 7), (1, 100 if dense else 11)]:
        fd, ok = fd_check(orc, P, pr, base, gu, gx, "Q", (0, t, j), 1e-4, rel_step=True)
        if ok:
            checked += 1
            assert abs(fd - g["dQ"][0, t, j]) <= 1e-6 * max(1, abs(fd)), ("Q", t, j)
    assert checked >= 12


def test_frozen_linearisation_fd_at_quadrotor_solution(orc, P):
    """Linearise the quadrotor at a converged nonlinear solution; the backward
    of the nonlinear solve must equal the FD gradient of the affine map."""
    import workloads as W
    d = W.make(0, B=1, T=6, pu_scale=0.01, seed=7)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=200, tol=1e-13)
    assert f["status"][0] & orc.ST_CONVERGED
    T = 6
    A = np.zeros((1, T, 13, 13))
    Bm = np.zeros((1, T, 13, 4))
    r = np.zeros((1, T, 13))
    for t in range(T - 1):
        A[0, t], Bm[0, t] = orc.rk4_jac(P, f["x"][0, t], f["u"][0, t])
        r[0, t] = orc.rk4(P, f["x"][0, t], f["u"][0, t]) - A[0, t] @ f["x"][0, t] - Bm[0, t] @ f["u"][0, t]
    pr = dict(affine=(A, Bm, r), x0=d["x0"].astype(np.float64), Q=d["Q"].astype(np.float64),
              p=d["p"].astype(np.float64), lo=d["lo"].astype(np.float64), hi=d["hi"].astype(np.float64))
    base = solve(orc, P, pr, u_init=f["u"])
    assert np.abs(base["u"] - f["u"]).max() < 1e-8  # (x*, u*) is a fixed point of the frozen model
    rng = np.random.default_rng(3)
    gu = rng.normal(size=(1, T, 4))
    gx = np.zeros((1, T, 13))
    g_nl = orc.backward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"], gu)
    checked = 0
    for (t, i) in [(0, 13), (1, 14), (2, 0), (3, 7), (4, 15), (5, 16)]:
        fd, ok = fd_check(orc, P, pr, base, gu, gx, "p", (0, t, i), 1e-6)
        if ok:
            checked += 1
            assert abs(fd - g_nl["dp"][0, t, i]) <= 1e-6 * max(1, abs(fd)), (t, i)
    for i in (0, 4, 9, 11):
        fd, ok = fd_check(orc, P, pr, base, gu, gx, "x0", (0, i), 1e-6)
        if ok:
            checked += 1
            assert abs(fd - g_nl["dx0"][0, i]) <= 1e-6 * max(1, abs(fd)), i
    assert checked >= 6


def test_structural_properties(orc, P):
    import workloads as W
    d = W.make(0)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    m = orc.active_mask(f["u"], d["lo"], d["hi"])
    rng = np.random.default_rng(0)
    g1 = rng.normal(size=d["grad_u"].shape)
    g2 = rng.normal(size=d["grad_u"].shape)
    args = (P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"])
    r1 = orc.backward(*args, g1)
    r2 = orc.backward(*args, g2)
    r12 = orc.backward(*args, 2.0 * g1 - 3.0 * g2)
    for k in ("dQ", "dp", "dx0"):  # linear in the upstream gradient
        assert np.allclose(r12[k], 2.0 * r1[k] - 3.0 * r2[k], rtol=1e-10, atol=1e-10)
    # dL/dc_u is zero on active controls
    for i in range(4):
        act = ((m >> i) & 1).astype(bool)
        assert np.all(r1["dp"][..., 13 + i][act] == 0.0)
    # every control active -> the solution does not depend on x_init
    allm = np.full_like(m, 15)
    r = orc.backward(*args, g1, mask=allm)
    assert np.all(r["dx0"] == 0.0)


def test_kkt_residuals_at_nonlinear_convergence(orc, P):
    """First-order KKT conditions of eq. (3) hold at a converged iLQR point:
    costates lam_t = C_x z_t + c_x + A_t^T lam_{t+1} (lam_{T} = 0), and the
    control gradient C_u z_t + c_u + B_t^T lam_{t+1} vanishes on free controls,
    is >= 0 at a lower bound and <= 0 at an upper bound."""
    import workloads as W
    d = W.make(0, B=4, T=8, pu_scale=0.01, seed=11)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=300, tol=1e-13)
    n_conv = 0
    for b in range(4):
        if not f["status"][b] & orc.ST_CONVERGED:
            continue
        n_conv += 1
        T = 8
        lam = np.zeros(13)
        scale = 1.0 + np.abs(d["p"][b]).max()
        for t in range(T - 1, -1, -1):
            z = np.concatenate([f["x"][b, t], f["u"][b, t]])
            C = np.diag(d["Q"][b, t].astype(np.float64))
            gz = C @ z + d["p"][b, t]
            if t < T - 1:
                A, Bm = orc.rk4_jac(P, f["x"][b, t], f["u"][b, t])
                gu = gz[13:] + Bm.T @ lam
                lam = gz[:13] + A.T @ lam
            else:
                gu = gz[13:]
                lam = gz[:13]
            for i in range(4):
                u = f["u"][b, t, i]
                if u == d["lo"][b, i]:
                    assert gu[i] >= -1e-8 * scale
                elif u == d["hi"][b, i]:
                    assert gu[i] <= 1e-8 * scale
                else:
                    assert abs(gu[i]) <= 1e-8 * scale, (b, t, i, gu[i])
    assert n_conv >= 2
