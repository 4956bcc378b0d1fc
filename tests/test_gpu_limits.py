"""GPU tests at the library's size limits: the longest horizon (T_max =
DMPC_T_LIMIT = 1024) in every launch form, with and without checkpointing,
and the largest iteration count (K = DMPC_K_LIMIT = 255, whose count fills
the status word's 8-bit field).  Parity against the FP64 oracle with the
kernel's decisions replayed, at the bars of the other parity tests."""
import numpy as np
import pytest

import workloads as W

from gpu_util import oracle_replay, rel, run_gpu
from test_gpu_parity import check_parity

pytestmark = pytest.mark.gpu

T_LIMIT, K_LIMIT = 1024, 255


@pytest.mark.parametrize("form", ["persistent", "plain", "tpar", "persistent_ckpt"])
def test_longest_horizon(form):
    d = W.make_hover_target(3, T_LIMIT, seed=4101, K=2)
    d["T"][1] = 700  # a ragged instance among full-length ones
    pad = np.arange(T_LIMIT)[None, :] >= d["T"][:, None]
    d["Q"][pad] = 0
    d["p"][pad] = 0
    d["grad_u"][pad] = 0
    kw = dict(plain=form == "plain", tpar=form == "tpar", ckpt=64 if form == "persistent_ckpt" else 0)
    g = run_gpu(d, **kw)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "T=1024 " + form)


def test_largest_iteration_count():
    d = W.make(0, B=8, T=10, pu_scale=0.01, seed=4102)
    d["K"] = K_LIMIT
    g = run_gpu(d, K=K_LIMIT, tol=0.0)
    iters = (g["status"] >> 8) & 255
    assert np.all(iters == K_LIMIT)
    o = oracle_replay(d, g)
    check_parity(d, g, o, "K=255")


def test_mpc_step_at_the_longest_horizon():
    import torch

    import paper_2605_29155_amd as D
    from gpu_util import handle
    import oracle as orc
    rng = np.random.default_rng(4103)
    B = 5
    us = rng.uniform(0, 8, size=(B, T_LIMIT, 4)).astype(np.float32)
    T = np.array([T_LIMIT, 1, 0, 513, T_LIMIT - 1], np.int32)
    x = W.hover_state(B).astype(np.float32)
    xs = torch.from_numpy(x).cuda()
    ust = torch.from_numpy(us).cuda()
    D.mpc_step(handle(), D.make_config(B, T_LIMIT), D.quad_params(W.quad_params_f32()), torch.from_numpy(T).cuda(),
               xs, ust, ust, None)
    torch.cuda.synchronize()
    assert np.array_equal(ust.cpu().numpy(), orc.shift_warm_start(us, T).astype(np.float32))
    assert rel(xs.cpu().numpy()[T > 0], np.stack([orc.rk4(orc.params_from(W.quad_params_f32()), x[b].astype(np.float64),
                                                          us[b, 0].astype(np.float64))
                                                  for b in range(B) if T[b] > 0])).max() <= 1e-5
