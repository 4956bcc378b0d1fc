"""The precision decisions of the GPU forward, shown on the CPU.

The GPU forward keeps the dynamics, the linearisation, the line search and
all storage in FP32, and accumulates the stage algebra (g, Y = V F,
Q = C + F^T Y, q, the value update) and the control block (its L D L^T
factorisation and the box-QP) in FP64.  precision_emulation.py replays the
decisions of a free FP64 oracle run with the precision of each step chosen
separately; its difference from that oracle run is the arithmetic alone.
These tests pin the emulation to the oracle and record what each choice costs
against the 1e-4 bar on u*:

  * FP32 accumulation of the stage algebra fails the bar;
  * an FP32 control block fails it too, on ordinary instances whose pivots
    are far above 1e-6, so an FP32 factorisation with an FP64 redo on small
    pivots only could not meet it either: the block is FP64 always;
  * holding V in FP32 between stages is harmless;
  * on long, unconverged horizons (T up to 50, 10 iterations) the kernel's
    FP32 dynamics carry the error past the bar on a few instances, and FP64
    dynamics would bring them back under it.
"""
import numpy as np
import pytest

import oracle as orc
import precision_emulation as E
import workloads as W

from gpu_util import rel

pytestmark = pytest.mark.slow

P = W.quad_params_f32()
P64 = orc.params_from(P)
BAR = 1e-4


def run(d, K, tol=0.0, idx=None):
    """Free FP64 oracle run on the instances idx; returns (sub-workload, its
    u*, its decisions)."""
    if idx is not None:
        d = {k: (v[idx] if isinstance(v, np.ndarray) and v.shape[:1] == (d["B"],) else v) for k, v in d.items()}
        d["B"] = len(idx)
    f = orc.forward(P64, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=K, tol=tol)
    return d, f["u"], (f["iters"], f["alpha"], f["pattern"])


def err(d, u_ref, dec, prec, stats=None):
    u, _ = E.forward(P, d, dec, prec, orc.alphas(), stats=stats)
    return rel(u, u_ref)


@pytest.fixture(scope="module")
def cfg1_32():
    return run(W.make(1, B=32, T=20), K=5)


def test_emulation_in_fp64_is_the_oracle():
    for d, K in ((W.make(0), 5), (W.make(1, B=8, T=20), 5), (W.make(1, B=4, T=50, seed=3003), 3)):
        d, u, dec = run(d, K)
        assert err(d, u, dec, E.ALL64).max() <= 1e-9


def test_kernel_precision_meets_the_bar(cfg1_32):
    for d, u, dec in (run(W.make(0), 5), cfg1_32):
        assert err(d, u, dec, E.KERNEL).max() <= 1e-5


def test_fp32_stage_accumulation_fails_the_bar(cfg1_32):
    d, u, dec = cfg1_32
    assert err(d, u, dec, E.variant(acc=E.f32)).max() > BAR
    assert err(d, u, dec, E.variant(acc=E.f32, vupd=E.f32)).max() > BAR


def test_fp32_control_block_fails_the_bar_without_small_pivots(cfg1_32):
    d, u, dec = cfg1_32
    stats = []
    e = err(d, u, dec, E.variant(fact=E.f32), stats)
    bad = np.nonzero(e > BAR)[0]
    assert len(bad) >= 1
    # the failing instances' smallest FP32 pivot is far above the 1e-6 at
    # which a fallback to FP64 would take over
    assert min(stats[b]["min_pivot"] for b in bad) > 1e-4


def test_fp32_value_function_storage_is_harmless(cfg1_32):
    d, u, dec = cfg1_32
    assert err(d, u, dec, E.variant(vstore=E.f32)).max() <= 1e-5


def test_long_unconverged_horizons_carried_by_fp32_dynamics():
    """Two instances of the ragged workload (T 49 and 47, 10 iterations, none
    converged) where the kernel's precision leaves u* past the bar; the
    linearisation alone or the rollout alone in FP64 is not enough, both
    together (with the trajectories) bring both under it."""
    d, u, dec = run(W.make(3), 10, 1e-5, idx=np.array([2368, 3968]))
    assert err(d, u, dec, E.KERNEL).max() > BAR
    assert err(d, u, dec, E.variant(lin=E.f64)).max() > BAR
    assert err(d, u, dec, E.variant(lin=E.f64, roll=E.f64, traj=E.f64)).max() <= BAR
    assert err(d, u, dec, E.ALL64).max() <= 1e-9
