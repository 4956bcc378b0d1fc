"""Pins of the oracle's stagewise box-QP (Sec. IV "Backward pass with input
bounds": the control update solves a box-constrained QP, after Tassa et al.).

The oracle enumerates the 3^4 clamp patterns.  It is pinned to the KKT
conditions of a strictly convex box-QP (which single out the unique
minimiser), to numpy's linear solve when no bound is active, to the separable
closed form for diagonal H, and to a projected-gradient solve.
"""
import numpy as np
import pytest


def rand_spd(rng, n=4, lo=0.05):
    M = rng.normal(size=(n, n))
    return M @ M.T + lo * np.eye(n)


def kkt_ok(H, q, a, b, d, tol=1e-9):
    g = H @ d + q
    scale = 1 + np.abs(q).max() + np.abs(H).max() * np.abs(d).max()
    for i in range(4):
        if d[i] < a[i] - tol or d[i] > b[i] + tol:
            return False
        at_lo, at_hi = abs(d[i] - a[i]) <= tol, abs(d[i] - b[i]) <= tol
        if at_lo and not at_hi and g[i] < -tol * scale:
            return False
        if at_hi and not at_lo and g[i] > tol * scale:
            return False
        if not at_lo and not at_hi and abs(g[i]) > tol * scale:
            return False
    return True


@pytest.mark.parametrize("seed", range(40))
def test_boxqp_satisfies_kkt(orc, seed):
    rng = np.random.default_rng(seed)
    H = rand_spd(rng)
    q = rng.normal(size=4) * 3
    a = -rng.uniform(0.1, 2, 4)
    b = rng.uniform(0.1, 2, 4)
    d, pat, st = orc.boxqp(H, q, a, b)
    assert st == 0
    assert kkt_ok(H, q, a, b, d)
    # the pattern is consistent with the solution
    for i in range(4):
        if pat[i] == orc.LOWER:
            assert d[i] == a[i]
        elif pat[i] == orc.UPPER:
            assert d[i] == b[i]


def test_unbounded_equals_linear_solve(orc):
    rng = np.random.default_rng(1)
    for _ in range(10):
        H = rand_spd(rng)
        q = rng.normal(size=4)
        d, pat, st = orc.boxqp(H, q, np.full(4, -1e30), np.full(4, 1e30))
        assert st == 0 and (pat == 0).all()
        ref = np.linalg.solve(H, -q)
        assert np.abs(d - ref).max() <= 1e-12 * max(1, np.abs(ref).max())


def test_diagonal_is_separable_clamp(orc):
    rng = np.random.default_rng(2)
    for _ in range(20):
        h = rng.uniform(0.01, 5, 4)
        q = rng.normal(size=4) * 2
        a, b = -np.ones(4), np.ones(4)
        d, pat, st = orc.boxqp(np.diag(h), q, a, b)
        assert np.abs(d - np.clip(-q / h, a, b)).max() <= 1e-13


def test_weakly_active_is_free(orc):
    # unconstrained optimum exactly on the upper bound (gradient 0 there)
    H = np.eye(4)
    b = np.array([1.0, 2.0, 0.5, 1.5])
    d, pat, st = orc.boxqp(H, -b, -np.ones(4), b)
    assert (pat == orc.FREE).all()
    assert np.array_equal(d, b)


def test_matches_projected_gradient(orc):
    rng = np.random.default_rng(5)
    for _ in range(10):
        H = rand_spd(rng, lo=0.5)
        q = rng.normal(size=4) * 2
        a, b = -np.ones(4), np.ones(4)
        d, _, _ = orc.boxqp(H, q, a, b)
        x = np.zeros(4)
        step = 1.0 / np.linalg.eigvalsh(H).max()
        for _ in range(20000):
            x = np.clip(x - step * (H @ x + q), a, b)
        assert np.abs(d - x).max() <= 1e-8


def test_nonfinite_input_flagged(orc):
    H = np.eye(4)
    q = np.array([np.nan, 0, 0, 0])
    d, pat, st = orc.boxqp(H, q, -np.ones(4), np.ones(4))
    assert st & orc.ST_NONFINITE


def test_lu_solve_matches_numpy(orc):
    rng = np.random.default_rng(9)
    M = rng.normal(size=(30, 30))
    r = rng.normal(size=30)
    assert np.allclose(orc.lu_solve(M, r), np.linalg.solve(M, r), rtol=1e-11, atol=1e-11)
