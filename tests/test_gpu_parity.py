"""GPU parity of the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (per-instance normwise relative error): 1e-4 on u*, 1e-3 on the
gradients dL/dQ, dL/dp, dL/dx0.  The oracle replays the kernel's discrete
decisions (line-search index, box-QP clamp patterns, iteration count, final
active set), each of which the kernel takes in FP32; the tests also check
that those decisions are valid for the oracle (the chosen candidate is a
minimiser up to rounding) and report how often a free FP64 run takes the same
ones.
"""
import numpy as np
import pytest

import workloads as W

from gpu_util import (TOL_G, TOL_U, alpha_choices_valid, decision_agreement, describe, oracle_replay,
                      parity_errors, rel, run_gpu, within_bars)

pytestmark = pytest.mark.gpu


def check_parity(d, g, o, label, check_grad=True):
    T = d["T"]
    e = parity_errors(g, o)
    if not check_grad:
        e.pop("g", None), e.pop("g_abs", None)
    ex = rel(g["x"], o["replay"]["x"])
    agree = decision_agreement(g, o)
    msg = "%s: %s | u* p99 %.2e | x* max %.2e | decisions agree %.4f" % (
        label, describe(e), np.percentile(e["u"], 99), ex.max(), agree)
    print(msg, flush=True)
    assert np.all(within_bars(e)), msg
    assert alpha_choices_valid(o) == 0
    # controls inside the box, padding zero
    lo, hi = d["lo"][:, None, :], d["hi"][:, None, :]
    assert np.all(g["u"] >= lo - 0) and np.all(g["u"] <= hi)
    pad = np.arange(d["T_max"])[None, :] >= T[:, None]
    assert np.all(g["u"][pad] == 0) and np.all(g["x"][pad] == 0)
    return agree


@pytest.mark.parametrize("plain", [False, True], ids=["persistent", "plain"])
def test_cfg0_parity(plain):
    d = W.make(0)
    g = run_gpu(d, plain=plain)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "cfg0 " + ("plain" if plain else "persistent"))
    assert g["launches_fwd"] == (3 * d["K"] + 4 if plain else 2)
    assert g["launches_bwd"] == 1


def test_cfg0_small_pu_parity():
    # p_u scaled by 0.01: non-trivial free sets in the box-QP
    d = W.make(0, pu_scale=0.01, seed=2000)
    g = run_gpu(d)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "cfg0 pu*0.01")


def test_ragged_edge_cases():
    # B not a multiple of 4; horizons 0, 1, 2 and T_max; tolerance-based stop
    d = W.make(3, B=7, T=12)
    d["T"] = np.array([0, 1, 2, 12, 5, 12, 3], np.int32)
    pad = np.arange(12)[None, :] >= d["T"][:, None]
    d["Q"][pad] = 0
    d["p"][pad] = 0
    d["grad_u"][pad] = 0
    g = run_gpu(d)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "ragged edge")
    assert g["status"][0] == 0 and np.all(g["dx0"][0] == 0) and np.all(g["dp"][0] == 0)


def test_cfg1_parity_full_size():
    d = W.make(1)
    g = run_gpu(d, need_grad=False)
    o = oracle_replay(d, g)
    agree = check_parity(d, g, o, "cfg1 B=1024 T=20", check_grad=False)
    assert agree >= 0.999


def test_persistent_equals_plain():
    d = W.make(1, B=64)
    a = run_gpu(d)
    b = run_gpu(d, plain=True)
    # same decisions; arithmetic differs only by where the linearisation is
    # formed (in-kernel vs a separate launch), so agreement is at rounding level
    assert np.array_equal(a["dlog"], b["dlog"])
    assert rel(a["u"], b["u"]).max() <= 1e-5
    assert rel(a["dp"], b["dp"]).max() <= 1e-4


def test_deterministic_and_lpt_invariant():
    d = W.make(3, B=64, T=20)
    a = run_gpu(d, lpt=True)
    b = run_gpu(d, lpt=True)
    c = run_gpu(d, lpt=False)
    for k in ("u", "x", "dQ", "dp", "dx0", "status", "dlog"):
        assert np.array_equal(a[k], b[k]), k
        assert np.array_equal(a[k], c[k]), k


def test_nonfinite_input_is_flagged():
    d = W.make(0, B=4)
    d["x0"][1, 0] = np.nan
    g = run_gpu(d)
    assert g["status"][1] & 0x4
    assert np.all(np.isfinite(g["u"][0])) and np.all(np.isfinite(g["u"][2]))


def test_fixed_control_bounds():
    # lo == hi on some rotors: those controls are always active
    d = W.make(0, B=4)
    d["lo"][:, 1] = 2.0
    d["hi"][:, 1] = 2.0
    g = run_gpu(d)
    assert np.all(g["u"][:, :, 1] == 2.0)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "fixed rotor")


def test_fp64_pivot_flag_and_tiny_control_weight():
    """Adversarial set: R scaled to 1e-8.  The control block is always
    factored in FP64, so fp64_pivot only decides which stages are flagged:
    the results are bitwise the same for every threshold, a threshold above
    every pivot flags every instance and a non-positive one flags none.
    Parity with the oracle at the conditioning-scaled bars (R = 1e-8 makes
    the stage QPs far more ill-conditioned than the workloads): an instance
    beyond the flat bars is held to them times s_b / 1e-5, where s_b is the
    FP64 oracle's own response to input noise at FP32 resolution (1e-7), so at
    most a hundred times the response."""
    from gpu_util import oracle_sensitivity
    d = W.make(0, B=64, r_scale=1e-6, seed=2006)
    a = run_gpu(d, fp64_pivot=1e-6)
    b = run_gpu(d, fp64_pivot=1e9)
    c = run_gpu(d, fp64_pivot=0.0)
    assert np.all((b["status"] & 0x8) != 0)
    assert not np.any(c["status"] & 0x8)
    for k in ("u", "x", "dQ", "dp", "dx0", "dlog"):
        assert np.array_equal(a[k], b[k]) and np.array_equal(a[k], c[k]), k
    o = oracle_replay(d, a)
    e = parity_errors(a, o)
    flat = within_bars(e)
    s = np.zeros(d["B"])
    if not flat.all():
        bad = np.nonzero(~flat)[0]
        s[bad] = oracle_sensitivity(d, o, idx=bad, orows=bad)
    scale = np.maximum(1.0, s / 1e-5)
    print("R=1e-8: flagged at 1e-6 %d/64 | %s | beyond the flat bars %d/64, their sensitivity max %.1e"
          % (np.sum((a["status"] & 0x8) != 0), describe(e), np.sum(~flat), s.max()), flush=True)
    assert np.all(within_bars(e, scale))
