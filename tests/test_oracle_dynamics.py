"""Pins of the oracle's quadrotor model and its RK4 Jacobian.

The paper never writes its drone model (Sec. V only names an agile drone), so
these tests pin the oracle to closed-form motions of the model this project
adopted (X-configuration, scalar-first quaternion, body rates) and pin the
analytic RK4 Jacobian (Sec. IV "Rollout and linearization": analytical A_t,
B_t) to the complex-step derivative of the oracle's own RK4 map.
"""
import numpy as np
import pytest


def hover(P):
    x = np.zeros(13)
    x[3] = 1.0
    return x, np.full(4, P.mass * P.g / 4.0)


def qmul(a, b):
    """Hamilton product, scalar first (textbook)."""
    aw, ax, ay, az = a
    bw, bx, by, bz = b
    return np.array([aw * bw - ax * bx - ay * by - az * bz,
                     aw * bx + ax * bw + ay * bz - az * by,
                     aw * by - ax * bz + ay * bw + az * bx,
                     aw * bz + ax * by - ay * bx + az * bw])


def test_hover_is_equilibrium(orc, P):
    x, u = hover(P)
    x[0:3] = [1.0, -2.0, 3.0]
    assert np.abs(orc.rk4(P, x, u) - x).max() <= 1e-15


def test_free_fall_is_exact(orc, P):
    # u = 0, w = 0, level: p(t) = p0 + v0 t - g t^2/2 e3 (RK4 is exact on this quadratic)
    x = np.zeros(13)
    x[3] = 1.0
    x[0:3] = [0.3, -0.1, 2.0]
    x[7:10] = [1.0, -0.5, 0.25]
    dt = P.dt
    for _ in range(5):
        x = orc.rk4(P, x, np.zeros(4))
    t = 5 * dt
    p = np.array([0.3, -0.1, 2.0]) + np.array([1.0, -0.5, 0.25]) * t - 0.5 * P.g * t * t * np.array([0, 0, 1])
    v = np.array([1.0, -0.5, 0.25]) - P.g * t * np.array([0, 0, 1])
    assert np.abs(x[0:3] - p).max() <= 1e-12
    assert np.abs(x[7:10] - v).max() <= 1e-12
    assert np.abs(x[3:7] - [1, 0, 0, 0]).max() == 0.0


@pytest.mark.parametrize("q0", [(1, 0, 0, 0), (0.8, 0.1, -0.3, 0.5)])
def test_torque_free_spin_about_z(orc, P, q0):
    # equal thrusts give no torque; w = (0,0,r) about a principal axis stays
    # constant, and body-rate kinematics give q(t) = q0 (x) (cos(rt/2), 0, 0, sin(rt/2))
    r = 2.0
    q0 = np.array(q0, float)
    q0 /= np.linalg.norm(q0)
    x = np.zeros(13)
    x[3:7] = q0
    x[12] = r
    u = np.full(4, 1.0)
    n = 20
    for _ in range(n):
        x = orc.rk4(P, x, u)
    t = n * P.dt
    qe = qmul(q0, np.array([np.cos(r * t / 2), 0, 0, np.sin(r * t / 2)]))
    # RK4 global error O((r dt)^4) per unit time; (r dt)^5 = 1e-5 per step
    assert np.abs(x[3:7] - qe).max() <= 1e-6
    assert np.abs(x[10:13] - [0, 0, r]).max() <= 1e-15


def test_tilted_thrust_direction(orc, P):
    # rotation by theta about body x: b3 = R e3 = (0, -sin th, cos th)
    th = 0.3
    x = np.zeros(13)
    x[3:7] = [np.cos(th / 2), np.sin(th / 2), 0, 0]
    u = np.full(4, 2.0)
    xd = orc.dyn(P, x, u)
    s = 8.0 / P.mass
    assert np.allclose(xd[7:10], [0, -s * np.sin(th), s * np.cos(th) - P.g], atol=1e-14, rtol=0)


def test_x_configuration_torque_signs(orc, P):
    # rotor 0 sits at (+a, +a): extra thrust on it gives tau = r x F = (a df, -a df, 0)
    # plus a yaw reaction kappa df (spin sign +1)
    x, u = hover(P)
    du = 0.1
    u2 = u.copy()
    u2[0] += du
    xd = orc.dyn(P, x, u2)
    a = P.arm / np.sqrt(2)
    assert np.isclose(xd[10], a * du / P.Jxx, rtol=1e-12)
    assert np.isclose(xd[11], -a * du / P.Jyy, rtol=1e-12)
    assert np.isclose(xd[12], P.kappa * du / P.Jzz, rtol=1e-12)
    # rotor 1 at (-a, +a), spin sign -1
    u3 = u.copy()
    u3[1] += du
    xd = orc.dyn(P, x, u3)
    assert np.isclose(xd[10], a * du / P.Jxx, rtol=1e-12)
    assert np.isclose(xd[11], a * du / P.Jyy, rtol=1e-12)
    assert np.isclose(xd[12], -P.kappa * du / P.Jzz, rtol=1e-12)


def test_constant_roll_torque_from_rest(orc, P):
    # w along a principal axis from rest under constant torque: w(t) = tau/J t (exact for RK4)
    x, u = hover(P)
    u = u + np.array([0.2, 0.2, -0.2, -0.2])  # pure roll torque, same total thrust
    a = P.arm / np.sqrt(2)
    tau = a * 0.8
    for _ in range(4):
        x = orc.rk4(P, x, u)
    assert np.isclose(x[10], tau / P.Jxx * 4 * P.dt, rtol=1e-12)
    assert abs(x[11]) < 1e-14 and abs(x[12]) < 1e-14


def test_gyroscopic_coupling(orc, P):
    # w x J w term: w = (1, 0, 1) gives w' _y = -(Jxx - Jzz) w_z w_x / Jyy
    x, u = hover(P)
    x[10], x[12] = 1.0, 1.0
    xd = orc.dyn(P, x, u)
    assert np.isclose(xd[11], -(P.Jxx - P.Jzz) / P.Jyy, rtol=1e-12)


@pytest.mark.parametrize("seed", range(6))
def test_rk4_jacobian_matches_complex_step(orc, P, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=13)
    if seed % 2 == 0:
        x[3:7] /= np.linalg.norm(x[3:7])  # also a non-unit quaternion on odd seeds
    x[10:13] *= 3.0
    u = rng.uniform(0.0, 8.5, size=4)
    A, B = orc.rk4_jac(P, x, u)
    J = np.hstack([A, B])
    cs = np.stack([orc.rk4_complex_step(P, x, u, np.eye(17)[j]) for j in range(17)], axis=1)
    assert np.abs(J - cs).max() <= 1e-12 * max(1.0, np.abs(cs).max())


def test_complex_step_matches_central_difference(orc, P):
    # the complex-step helper itself against plain central differences of rk4
    rng = np.random.default_rng(7)
    x = rng.normal(size=13)
    u = rng.uniform(0, 8, 4)
    h = 1e-6
    for j in (0, 4, 8, 11, 14):
        e = np.eye(17)[j]
        fd = (orc.rk4(P, x + h * e[:13], u + h * e[13:]) - orc.rk4(P, x - h * e[:13], u - h * e[13:])) / (2 * h)
        cs = orc.rk4_complex_step(P, x, u, e)
        assert np.abs(fd - cs).max() <= 1e-6 * max(1, np.abs(cs).max())


def test_trivial_jacobian_columns(orc, P):
    # nothing depends on p; v enters only through p' = v: dp/dv = dt I, dv/dv = I
    rng = np.random.default_rng(3)
    x = rng.normal(size=13)
    u = rng.uniform(0, 8, 4)
    A, _ = orc.rk4_jac(P, x, u)
    assert np.abs(A[:, 0:3] - np.eye(13)[:, 0:3]).max() <= 1e-15
    E = np.zeros((13, 3))
    E[0:3] = P.dt * np.eye(3)
    E[7:10] = np.eye(3)
    assert np.abs(A[:, 7:10] - E).max() <= 1e-15
    assert np.abs(A[10:13, 0:10]).max() == 0.0
