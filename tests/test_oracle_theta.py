"""Pins of the oracle's gradient with respect to the model constants
theta = (mass, Jxx, Jyy, Jzz, arm, kappa, dt, g).

The backward differentiates the LQ problem of the model linearised at the
solution (Sec. IV after eq. (3), after Amos et al. 2018).  theta enters that
problem through F_t = df/dz(z*_t; theta) and f_t = f(z*_t; theta) - F_t z*_t,
so:
  * central finite differences of the frozen-linearisation LQ solve (built
    from the RK4 map and its Jacobian at perturbed constants, active set held)
    must give the same gradient, with no costate or second derivative in it;
  * at the hover equilibrium with a cost whose gradient vanishes there, the
    costates of the solution are zero, the LQ Hessian is the exact Lagrangian
    Hessian, and the gradient equals finite differences of the full nonlinear
    solve;
  * gravity enters one RK4 step in closed form (constant acceleration is
    integrated exactly): d v_z / d g = -dt, d p_z / d g = -dt^2 / 2.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as W

from test_oracle_grad import fd_check, loss, mask, solve

NAMES = orc.THETA_NAMES


def with_param(P, j, v):
    vals = [getattr(P, n) for n in NAMES]
    vals[j] = v
    return orc.params(*vals)


def frozen_problem(P, f, d, T):
    A = np.zeros((1, T, 13, 13))
    Bm = np.zeros((1, T, 13, 4))
    r = np.zeros((1, T, 13))
    for t in range(T - 1):
        A[0, t], Bm[0, t] = orc.rk4_jac(P, f["x"][0, t], f["u"][0, t])
        r[0, t] = orc.rk4(P, f["x"][0, t], f["u"][0, t]) - A[0, t] @ f["x"][0, t] - Bm[0, t] @ f["u"][0, t]
    return dict(affine=(A, Bm, r), x0=d["x0"].astype(np.float64), Q=d["Q"].astype(np.float64),
                p=d["p"].astype(np.float64), lo=d["lo"].astype(np.float64), hi=d["hi"].astype(np.float64))


@pytest.mark.parametrize("seed", [7, 8])
def test_theta_gradient_matches_fd_of_the_frozen_linearisation(P, seed):
    T = 6
    d = W.make(0, B=1, T=T, pu_scale=0.01, seed=seed)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=200, tol=1e-13)
    assert f["status"][0] & orc.ST_CONVERGED
    rng = np.random.default_rng(seed)
    gu = rng.normal(size=(1, T, 4))
    gx = rng.normal(size=(1, T, 13))
    g = orc.backward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"], gu, gx, dtheta=True)
    base = solve(orc, P, frozen_problem(P, f, d, T), u_init=f["u"])
    m0 = mask(orc, base, d)
    checked = 0
    for j in range(orc.NTHETA):
        th = getattr(P, NAMES[j])
        hstep = 1e-4 * abs(th)
        vals, same = [], True
        for s in (+1, -1):
            Pj = with_param(P, j, th + s * hstep)
            fs = solve(orc, P, frozen_problem(Pj, f, d, T), u_init=f["u"])
            vals.append(loss(fs, gu, gx)[0])
            same &= np.array_equal(mask(orc, fs, d), m0)
        if not same:
            continue
        fd = (vals[0] - vals[1]) / (2 * hstep)
        scale = max(1.0, abs(fd), 1e-3 * np.abs(g["dtheta"][0]).max())
        assert abs(fd - g["dtheta"][0, j]) <= 1e-6 * scale, (NAMES[j], fd, g["dtheta"][0, j])
        checked += 1
    assert checked == orc.NTHETA


def test_theta_gradient_at_hover_matches_fd_of_the_nonlinear_solve(P):
    """At hover with target at the start state the solution is hover itself
    and its costates vanish; the LQ derivative is then the exact derivative of
    the converged nonlinear solution map."""
    B, T = 1, 8
    x0 = W.hover_state(B)
    hov = P.mass * P.g / 4
    Cd = np.r_[[10.0] * 3, [1.0] * 4, [1.0] * 3, [0.1] * 3, [0.01] * 4]
    zref = np.r_[np.zeros(3), 1.0, np.zeros(9), [hov] * 4]
    Q = np.broadcast_to(Cd, (B, T, 17)).copy()
    p = -(Q * zref)
    lo, hi = np.zeros((B, 4)), np.full((B, 4), 8.5)
    f = orc.forward(P, x0, Q, p, lo, hi, K=100, tol=1e-14)
    assert np.abs(f["u"] - hov).max() < 1e-12
    rng = np.random.default_rng(5)
    gu = rng.normal(size=(B, T, 4))
    gx = rng.normal(size=(B, T, 13))
    g = orc.backward(P, x0, Q, p, lo, hi, f["u"], f["x"], gu, gx, dtheta=True)["dtheta"][0]
    fd = np.zeros(orc.NTHETA)
    for j in range(orc.NTHETA):
        th = getattr(P, NAMES[j])
        hstep = 1e-5 * abs(th)
        v = []
        for s in (+1, -1):
            Pj = with_param(P, j, th + s * hstep)
            fj = orc.forward(Pj, x0, Q, p, lo, hi, K=100, tol=1e-14)
            assert fj["status"][0] & orc.ST_CONVERGED
            v.append(np.sum(fj["u"] * gu) + np.sum(fj["x"] * gx))
        fd[j] = (v[0] - v[1]) / (2 * hstep)
    scale = np.abs(fd).max()
    assert scale > 1e-2  # mass and g move the hover thrust
    assert np.abs(g - fd).max() <= 1e-6 * scale, (g, fd)


def test_gravity_enters_one_step_in_closed_form(P):
    """With only the upstream gradient on x*_1 (v_z, p_z) and every control
    held at a bound, the solution's response to g is one RK4 step's."""
    B, T = 1, 2
    rng = np.random.default_rng(2)
    x0 = W.hover_state(B) + 0.1 * rng.normal(size=(B, 13))
    Q = np.full((B, T, 17), 1.0)
    p = np.zeros((B, T, 17))
    p[..., 13:] = -50.0  # pushes every control to the upper bound
    lo, hi = np.zeros((B, 4)), np.full((B, 4), 3.0)
    f = orc.forward(P, x0, Q, p, lo, hi, K=20, tol=1e-14)
    assert np.all(f["u"] == 3.0)
    gu = np.zeros((B, T, 4))
    gx = np.zeros((B, T, 13))
    gx[0, 1, 9] = 1.0   # dL/dv_z(1)
    gx[0, 1, 2] = 0.5   # dL/dp_z(1)
    g = orc.backward(P, x0, Q, p, lo, hi, f["u"], f["x"], gu, gx, dtheta=True)["dtheta"][0]
    dt = P.dt
    assert abs(g[7] - (-dt - 0.5 * dt * dt / 2)) <= 1e-12


def test_theta_gradient_structure(P):
    d = W.make(0, B=4, T=7, seed=21)
    f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=5)
    rng = np.random.default_rng(1)
    g1, g2 = rng.normal(size=(2,) + d["grad_u"].shape)
    args = (P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"])
    r1 = orc.backward(*args, g1, dtheta=True)["dtheta"]
    r2 = orc.backward(*args, g2, dtheta=True)["dtheta"]
    r12 = orc.backward(*args, 2.0 * g1 - 3.0 * g2, dtheta=True)["dtheta"]
    # linear in the upstream gradient: lt and zt are, and the solution's own
    # costates only multiply zt
    assert np.allclose(r12, 2.0 * r1 - 3.0 * r2, rtol=1e-9, atol=1e-9 * np.abs(r12).max())
    assert np.all(orc.backward(*args, 0.0 * g1, dtheta=True)["dtheta"] == 0.0)
    # a one-stage horizon has no dynamics step
    T1 = np.array([1, 1, 1, 1], np.int32)
    f1 = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], T1, K=5)
    r = orc.backward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f1["u"], f1["x"], g1, T=T1, dtheta=True)
    assert np.all(r["dtheta"] == 0.0)
    # the two backward methods carry the same dtheta (it depends only on zt)
    rk = orc.backward(*args, g1, method=1, dtheta=True)["dtheta"]
    assert np.allclose(rk, r1, rtol=1e-8, atol=1e-8 * np.abs(r1).max())
