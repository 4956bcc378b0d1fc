"""Pins of the oracle's receding-horizon loop (Sec. III-A; the outer loops of Alg. 1 and Alg. 2:
solve from the current state, apply the first control, repeat from the state
reached) and of its shifted warm start.

  * hover is an equilibrium of the quadrotor (eq. (1)): with the target at
    the start state the closed loop must stay there, applying m g / 4;
  * on time-invariant affine dynamics without active bounds the horizon
    problem is a finite-horizon LQR, so the closed loop is x <- (A + B K_0) x
    with K_0 from the textbook Riccati difference equation;
  * in the nominal loop (plant = model) the shifted solution rolled out from
    the state reached reproduces the tail of the previous optimal trajectory;
  * a warm start changes where the iteration starts, not where it converges.
"""
import numpy as np
import pytest

import oracle as orc
import workloads as W

P = orc.params_from(W.quad_params_f32())


def hover_problem(B, T):
    x0 = W.hover_state(B)
    hov = P.mass * P.g / 4
    C = np.r_[[10.0] * 3, [1.0] * 4, [1.0] * 3, [0.1] * 3, [0.01] * 4]
    zref = np.r_[np.zeros(3), 1.0, np.zeros(9), [hov] * 4]
    Q = np.broadcast_to(C, (B, T, 17)).copy()
    p = -(Q * zref)
    return x0, Q, p, np.zeros((B, 4)), np.full((B, 4), 8.5)


@pytest.mark.parametrize("warm", [True, False])
def test_hover_is_a_fixed_point_of_the_closed_loop(warm):
    x0, Q, p, lo, hi = hover_problem(3, 10)
    r = orc.receding_horizon(P, x0, (Q, p), lo, hi, 6, K=5, warm=warm)
    assert np.abs(r["x"] - x0[None]).max() <= 1e-12
    assert np.abs(r["u"] - P.mass * P.g / 4).max() <= 1e-9


def textbook_lqr_gain(A, B, Qx, R, T):
    """First gain of the finite-horizon LQR with T controls: the last control
    only pays its own weight, so P_{T-1} = Qx; then the Riccati difference
    equation backwards to t = 0."""
    Pm = Qx.copy()
    K = None
    for _ in range(T - 1):
        S = R + B.T @ Pm @ B
        K = -np.linalg.solve(S, B.T @ Pm @ A)
        Pm = Qx + A.T @ Pm @ A + A.T @ Pm @ B @ K
    return K


@pytest.mark.parametrize("warm", [True, False])
def test_affine_closed_loop_is_receding_horizon_lqr(warm):
    rng = np.random.default_rng(41)
    nb, T, steps = 3, 8, 6
    A = np.eye(13) + 0.1 * rng.normal(size=(13, 13))
    Bm = 0.3 * rng.normal(size=(13, 4))
    qx = 10 ** rng.uniform(-1, 1, size=13)
    ru = rng.uniform(0.05, 0.5, size=4)
    Q = np.broadcast_to(np.r_[qx, ru], (nb, T, 17)).copy()
    p = np.zeros((nb, T, 17))
    aff = (np.broadcast_to(A, (nb, T, 13, 13)).copy(), np.broadcast_to(Bm, (nb, T, 13, 4)).copy(),
           np.zeros((nb, T, 13)))
    x0 = rng.normal(size=(nb, 13))
    lo, hi = np.full((nb, 4), -1e30), np.full((nb, 4), 1e30)
    r = orc.receding_horizon(P, x0, (Q, p), lo, hi, steps, K=1, warm=warm, affine=aff,
                             plant=lambda x, u: x @ A.T + u @ Bm.T)
    K0 = textbook_lqr_gain(A, Bm, np.diag(qx), np.diag(ru), T)
    x = x0.copy()
    for k in range(steps):
        u = x @ K0.T
        assert np.allclose(r["u"][k], u, rtol=1e-9, atol=1e-9 * np.abs(u).max())
        x = x @ A.T + u @ Bm.T
        assert np.allclose(r["x"][k + 1], x, rtol=1e-9, atol=1e-9 * np.abs(x).max())


def test_shifted_warm_start_reproduces_the_previous_tail():
    d = W.make_hover_target(4, 10, seed=7)
    x0, Q, p, lo, hi = (d[k].astype(np.float64) for k in ("x0", "Q", "p", "lo", "hi"))
    r = orc.receding_horizon(P, x0, (Q, p), lo, hi, 4, K=5, warm=True)
    for k in range(3):
        u0 = orc.shift_warm_start(r["u_star"][k])
        roll = orc.forward(P, r["x"][k + 1], Q, p, lo, hi, K=0, u_init=u0)
        # stage 0 of the new rollout is the state reached; stages 1..T-2 follow
        # the previous optimal trajectory from its stage 2 on
        assert np.abs(roll["x"][:, :-1] - r["x_star"][k][:, 1:]).max() <= 1e-12
        assert np.array_equal(roll["u"], np.clip(u0, lo[:, None], hi[:, None]))


def test_warm_start_keeps_the_optimum_and_saves_iterations():
    d = W.make_hover_target(6, 20, seed=5)
    x0, Q, p, lo, hi = (d[k].astype(np.float64) for k in ("x0", "Q", "p", "lo", "hi"))
    rw = orc.receding_horizon(P, x0, (Q, p), lo, hi, 8, K=40, tol=1e-9, warm=True)
    rc = orc.receding_horizon(P, x0, (Q, p), lo, hi, 8, K=40, tol=1e-9, warm=False)
    assert np.abs(rw["u_star"] - rc["u_star"]).max() <= 1e-6
    assert np.abs(rw["x"] - rc["x"]).max() <= 1e-6
    # the first solve is cold in both runs; every later one starts closer
    assert np.array_equal(rw["iters"][0], rc["iters"][0])
    assert rw["iters"][1:].sum() < 0.9 * rc["iters"][1:].sum()


def test_shift_definition_on_ragged_horizons():
    rng = np.random.default_rng(3)
    u = rng.normal(size=(5, 6, 4))
    T = np.array([6, 3, 1, 0, 2], np.int32)
    s = orc.shift_warm_start(u, T)
    for b, tb in enumerate(T):
        exp = np.zeros((6, 4))
        if tb > 0:
            exp[:tb] = np.concatenate([u[b, 1:tb], u[b, tb - 1:tb]])
        assert np.array_equal(s[b], exp)


def test_empty_horizon_keeps_its_state():
    x0, Q, p, lo, hi = hover_problem(2, 6)
    x0[:, 7] = 0.5  # moving, so a step would change the state
    r = orc.receding_horizon(P, x0, (Q, p), lo, hi, 3, T=np.array([6, 0], np.int32), K=3)
    assert np.array_equal(r["x"][:, 1], np.broadcast_to(x0[1], (4, 13)))
    assert np.all(r["u"][:, 1] == 0)
    assert np.abs(r["x"][1, 0] - x0[0]).max() > 1e-3


@pytest.mark.parametrize("mutant", ["applies_stage_1", "unshifted_warm_start", "state_not_advanced"])
def test_pins_catch_planted_loop_mistakes(mutant, monkeypatch):
    """Each plausible mistake in the loop, planted in a copy of the oracle's
    own source, fails at least one of the pins above."""
    import inspect
    src = inspect.getsource(orc.receding_horizon)
    old, new = {
        "applies_stage_1": ('out["u"][:, 0].copy()', 'out["u"][:, 1].copy()'),
        "unshifted_warm_start": ('shift_warm_start(out["u"], Tb) if warm else None', 'out["u"] if warm else None'),
        "state_not_advanced": ("x = np.where(live[:, None], xn, x)", "x = x"),
    }[mutant]
    assert src.count(old) == 1
    ns = {}
    exec(src.replace(old, new), orc.__dict__, ns)
    monkeypatch.setattr(orc, "receding_horizon", ns["receding_horizon"])
    pins = [lambda: test_hover_is_a_fixed_point_of_the_closed_loop(True),
            lambda: test_affine_closed_loop_is_receding_horizon_lqr(True),
            test_shifted_warm_start_reproduces_the_previous_tail,
            test_warm_start_keeps_the_optimum_and_saves_iterations,
            test_empty_horizon_keeps_its_state]
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed >= 1
