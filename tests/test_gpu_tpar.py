"""GPU tests of the per-launch form with the time-parallel Riccati
(DMPC_TPAR): the backward pass of each iteration is an associative scan over
the stages under the previous iteration's clamp pattern, checked stage by
stage, with the serial sweep as fallback.  It computes the same iteration as
the serial form, so the same oracle (decisions replayed) and bars apply:
1e-4 on u*, 1e-3 on the gradients."""
import numpy as np
import pytest

import workloads as W

from gpu_util import oracle_replay, rel, run_gpu
from test_gpu_parity import check_parity

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", ["cfg0", "cfg0_free", "hover_b1_t50", "hover_b16_t50", "ragged", "dense",
                                  "ckpt"])
def test_tpar_matches_oracle(case):
    if case == "cfg0":
        d = W.make(0)
    elif case == "cfg0_free":
        d = W.make(0, B=32, T=16, pu_scale=0.01, seed=3101)
    elif case == "hover_b1_t50":
        d = W.make_hover_target(1, 50, seed=3102)
    elif case == "hover_b16_t50":
        d = W.make_hover_target(16, 50, seed=3103)
    elif case == "ragged":
        d = W.make(3, B=7, T=12, seed=3104)
        d["T"] = np.array([0, 1, 2, 12, 5, 12, 3], np.int32)
        pad = np.arange(12)[None, :] >= d["T"][:, None]
        d["Q"][pad] = 0
        d["p"][pad] = 0
        d["grad_u"][pad] = 0
    elif case == "dense":
        d = W.make(4, B=16, T=12, seed=3105)
    else:
        d = W.make(0, B=16, T=14, pu_scale=0.01, seed=3108)
    g = run_gpu(d, tpar=True, ckpt=4 if case == "ckpt" else 0)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "tpar " + case)


def test_tpar_agrees_with_the_serial_form():
    """Same decisions as the serial per-launch form and the same solution to
    rounding (the scanned value functions differ from the serial ones only in
    FP64 rounding order)."""
    d = W.make_hover_target(8, 40, seed=3106)
    a = run_gpu(d, plain=True)
    b = run_gpu(d, plain=True, tpar=True)
    assert np.array_equal(a["dlog"], b["dlog"])
    assert rel(a["u"], b["u"]).max() <= 1e-5
    assert rel(a["dp"], b["dp"]).max() <= 1e-4


def test_tpar_launch_structure():
    d = W.make_hover_target(2, 20, seed=3107)
    g = run_gpu(d, tpar=True)
    levels = 5  # ceil(log2 20)
    # init; per iteration lin, elements, levels, gains, fallback sweep, line search; the tail through the
    # same scan (lin, elements, levels, factors); outputs
    assert g["launches_fwd"] == 1 + d["K"] * (1 + 1 + levels + 1 + 2) + (levels + 3) + 1
    # with checkpointing the tail is the serial sweep
    g = run_gpu(d, tpar=True, ckpt=4)
    assert g["launches_fwd"] == 1 + d["K"] * (1 + 1 + levels + 1 + 2) + 2 + 1


def test_tpar_needs_its_workspace():
    import ctypes as C

    import torch

    import paper_2605_29155_amd as D
    from gpu_util import handle
    h = handle()
    B, T = 4, 10
    cfg = D.make_config(B, T, 0, 3, 0.0, D.TUNED)
    D.set_tuned(h, cfg, False, D.LaunchChoice(2, 0, 1, 0, 0.0))
    ws = D.alloc_workspace(cfg, "cuda:0")
    d = W.make_hover_target(B, T)
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to("cuda:0") for k in ("x0", "Q", "p", "lo", "hi")}
    u = torch.zeros(B, T, 4, device="cuda:0")
    st = torch.zeros(B, dtype=torch.int32, device="cuda:0")
    with pytest.raises(D.DMPCError, match="EWORKSPACE"):
        D.forward_raw(h, cfg, D.quad_params(W.quad_params_f32()), t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None,
                      u, None, st, ws)
    torch.cuda.synchronize()
    del C
