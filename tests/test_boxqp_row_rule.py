"""The selection rule of the kernel's row-parallel box-QP (the stagewise QP of
Sec. IV, "Backward pass with input bounds"), modelled in numpy and checked
against the oracle's enumeration of the 3^4 clamp patterns.

The kernel's 16 lanes each take one free/clamped split (bit a of the lane
index set: coordinate a free) with every clamped coordinate on a guessed
bound, solve the face problem, and keep the lanes whose solution satisfies the
optimality conditions; the row takes the lowest valid lane.  Bounds are
guessed from the clamped warm start (the bound it sits on, else the side its
gradient points to), then, for rows with no valid lane, from the
unconstrained minimiser (the bound it lies beyond, else the first guess); the
rest fall back to the active-set method.  What the rule relies on, checked
here for strictly convex QPs:

  - a valid lane's face solution is the enumeration's minimiser (so the
    choice among several valid lanes cannot change the step beyond rounding);
  - on non-degenerate problems exactly one lane is valid when the guessed
    bounds are right, and none when a clamped coordinate's bound is wrong;
  - the two guesses cover the minimiser's bounds in most problems drawn like
    the stage QPs, and the unconstrained minimiser alone would not.

This models the rule, not the kernel's arithmetic; the kernel's outputs are
compared with the oracle by the GPU parity tests."""
import numpy as np
import pytest


def rand_spd(rng, n=4, lo=0.05):
    M = rng.normal(size=(n, n))
    return M @ M.T + lo * np.eye(n)


def face_solve(H, q, lo, hi, free, onlo, xfix=None):
    """Minimiser on the face: clamped coordinates on their guessed bound (a
    fixed coordinate, lo >= hi, at xfix), the free ones from the free block's
    linear system."""
    xc = np.where(onlo, lo, hi)
    if xfix is not None:
        xc = np.where(lo >= hi, xfix, xc)
    x = xc.copy()
    f = np.flatnonzero(free)
    if len(f):
        c = np.flatnonzero(~free)
        rhs = -(q[f] + H[np.ix_(f, c)] @ xc[c])
        x[f] = np.linalg.solve(H[np.ix_(f, f)], rhs)
    return x


def valid(H, q, lo, hi, free, onlo, x):
    g = H @ x + q
    fixed = ~(lo < hi)
    ok_free = (x >= lo) & (x <= hi)
    ok_clamped = np.where(onlo, g >= 0.0, g <= 0.0)
    ok = np.where(fixed, ~free, np.where(free, ok_free, ok_clamped))
    return bool(np.all(ok))


def lanes(H, q, lo, hi, onlo, xfix=None):
    """(lane, solution) for every valid lane, lowest first."""
    out = []
    for j in range(16):
        free = np.array([(j >> a) & 1 for a in range(4)], bool)
        x = face_solve(H, q, lo, hi, free, onlo, xfix)
        if valid(H, q, lo, hi, free, onlo, x):
            out.append((j, x))
    return out


def first_guess(H, q, lo, hi, xw):
    x0 = np.clip(xw, lo, hi)
    g0 = H @ x0 + q
    return (x0 <= lo) | (~(x0 >= hi) & (g0 > 0.0))


def row_solve(H, q, lo, hi, xw):
    """The rule: (step, pass that found it: 1, 2, or 0 for the fallback)."""
    onlo = first_guess(H, q, lo, hi, xw)
    v = lanes(H, q, lo, hi, onlo)
    if v:
        return v[0][1], 1
    xu = np.linalg.solve(H, -q)  # lane 15's solution: every coordinate free
    onlo = (xu < lo) | (~(xu > hi) & onlo)
    v = lanes(H, q, lo, hi, onlo)
    if v:
        return v[0][1], 2
    return None, 0


def stage_like(rng):
    """A QP shaped like the stage QPs: thrust-step bounds [0 - u, 8.5 - u]
    around a nominal thrust u in [0, 8.5], a curvature of mixed scale, a
    linear term that often pushes past a bound, and a warm start that is a
    perturbed solution (the previous iteration's step)."""
    H = rand_spd(rng) * 10.0 ** rng.uniform(-2, 1)
    u = rng.uniform(0.0, 8.5, 4)
    lo, hi = -u, 8.5 - u
    q = rng.normal(size=4) * 10.0 ** rng.uniform(-1, 1.5)
    xw = np.clip(rng.normal(size=4) * 2.0, lo, hi) if rng.uniform() < 0.8 else np.zeros(4)
    return H, q, lo, hi, xw


@pytest.mark.parametrize("seed", range(4))
def test_valid_lanes_give_the_enumerated_minimiser(orc, seed):
    rng = np.random.default_rng(7000 + seed)
    found = 0
    for _ in range(300):
        H, q, lo, hi, xw = stage_like(rng)
        ref, _, st = orc.boxqp(H, q, lo, hi)
        assert st == 0
        for guess in (first_guess(H, q, lo, hi, xw), rng.uniform(size=4) < 0.5):
            for j, x in lanes(H, q, lo, hi, guess):
                found += 1
                assert np.abs(x - ref).max() <= 1e-9 * (1 + np.abs(ref).max()), (j, x, ref)
    assert found > 300


def test_one_valid_lane_with_the_right_bounds_none_with_a_wrong_one(orc):
    rng = np.random.default_rng(7100)
    checked = 0
    for _ in range(400):
        H, q, lo, hi, _ = stage_like(rng)
        ref, pat, _ = orc.boxqp(H, q, lo, hi)
        clamped = pat != orc.FREE
        # skip degenerate problems (a clamped coordinate with a zero
        # multiplier, or a free one on a bound)
        g = H @ ref + q
        if np.any(clamped & (np.abs(g) < 1e-9)) or np.any(~clamped & ((np.abs(ref - lo) < 1e-9) | (np.abs(ref - hi) < 1e-9))):
            continue
        right = np.where(clamped, pat == orc.LOWER, rng.uniform(size=4) < 0.5)
        v = lanes(H, q, lo, hi, right)
        assert len(v) == 1
        j = v[0][0]
        assert all(bool((j >> a) & 1) == (not clamped[a]) for a in range(4))
        if clamped.any():
            wrong = right.copy()
            a = np.flatnonzero(clamped)[0]
            wrong[a] = not wrong[a]
            assert lanes(H, q, lo, hi, wrong) == []
        checked += 1
    assert checked > 300


def test_two_guesses_cover_most_stage_qps(orc):
    rng = np.random.default_rng(7200)
    n = 2000
    passes = np.zeros(3, int)
    unconstrained_only = 0
    for _ in range(n):
        H, q, lo, hi, xw = stage_like(rng)
        x, p = row_solve(H, q, lo, hi, xw)
        passes[p] += 1
        ref, pat, _ = orc.boxqp(H, q, lo, hi)
        if p:
            assert np.abs(x - ref).max() <= 1e-9 * (1 + np.abs(ref).max())
        xu = np.linalg.solve(H, -q)
        if not lanes(H, q, lo, hi, xu < lo):
            unconstrained_only += 1
    print("first guess %d, second %d, fallback %d of %d; bounds from the unconstrained minimiser alone miss %d"
          % (passes[1], passes[2], passes[0], n, unconstrained_only))
    assert passes[0] <= 0.08 * n
    assert passes[1] >= 0.7 * n
    assert unconstrained_only > passes[0]


def test_fixed_coordinates_are_never_free(orc):
    """A coordinate with lo = hi (a rotor whose thrust is pinned) is held on
    its bound in every lane and the lanes that would free it are invalid; the
    valid lane is still the enumeration's minimiser."""
    rng = np.random.default_rng(7300)
    seen = 0
    for _ in range(300):
        H, q, lo, hi, xw = stage_like(rng)
        a = rng.integers(0, 4)
        hi[a] = lo[a]
        ref, _, st = orc.boxqp(H, q, lo, hi)
        assert st == 0
        x0 = np.clip(xw, lo, hi)
        onlo = first_guess(H, q, lo, hi, xw)
        for j, x in lanes(H, q, lo, hi, onlo, xfix=x0):
            assert not (j >> a) & 1
            assert x[a] == lo[a]
            assert np.abs(x - ref).max() <= 1e-9 * (1 + np.abs(ref).max())
            seen += 1
    assert seen > 150
