"""GPU tests of the autotuner: every persistent launch choice computes the
same bits, the tuner stores and reuses its choice per shape, and a forward
with DMPC_TUNED launches what was chosen."""
import numpy as np
import pytest

import workloads as W

from gpu_util import handle, rel

pytestmark = pytest.mark.gpu


def _bufs(d, cfg, dev):
    import torch

    import paper_2605_29155_amd as D
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi", "grad_u")}
    t["T"] = torch.from_numpy(d["T"].astype(np.int32)).to(dev)
    B, Tm = d["B"], d["T_max"]
    o = dict(u=torch.zeros(B, Tm, 4, device=dev), x=torch.zeros(B, Tm, 13, device=dev),
             st=torch.zeros(B, dtype=torch.int32, device=dev), ws=D.alloc_workspace(cfg, dev),
             dl=torch.zeros(B, cfg.max_iter, 1 + Tm, dtype=torch.uint8, device=dev),
             gQ=torch.zeros_like(t["Q"]), gp=torch.zeros_like(t["p"]), gx0=torch.zeros_like(t["x0"]))
    return t, o


def _run(D, h, cfg, par, t, o):
    import torch
    D.forward_raw(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], t["T"], o["u"], o["x"], o["st"], o["ws"],
                  o["dl"])
    D.backward_raw(h, cfg, par, t["Q"], t["p"], t["lo"], t["hi"], o["ws"], t["grad_u"], None, o["gQ"], o["gp"],
                   o["gx0"])
    torch.cuda.synchronize()
    return {k: o[k].cpu().numpy().copy() for k in ("u", "x", "st", "dl", "gQ", "gp", "gx0")}


def test_every_persistent_choice_is_bitwise_identical():
    import paper_2605_29155_amd as D
    d = W.make(3, B=96, T=20, seed=5003)
    dev = "cuda:0"
    h = handle()
    cfg = D.make_config(96, 20, 0, 4, 1e-5, D.NEED_GRAD | D.TUNED)
    par = D.quad_params(W.quad_params_f32())
    t, o = _bufs(d, cfg, dev)
    ref = None
    for occ in (1, 2):
        for grid in (0, 1):
            for lpt in (0, 1):
                ch = D.LaunchChoice(0, lpt, occ, grid, 0.0)
                D.set_tuned(h, cfg, True, ch)
                r = _run(D, h, cfg, par, t, o)
                used = D.last_launch_choice(h)
                assert (used.plain, used.lpt, used.waves_per_simd, used.grid_mode) == (0, lpt, occ, grid)
                if ref is None:
                    ref = r
                for k in r:
                    assert np.array_equal(r[k], ref[k]), (occ, grid, lpt, k)
    # the per-launch form agrees to rounding
    D.set_tuned(h, cfg, True, D.LaunchChoice(1, 0, 1, 0, 0.0))
    r = _run(D, h, cfg, par, t, o)
    assert D.last_launch_choice(h).plain == 1
    du, dg = rel(r["u"], ref["u"]).max(), rel(r["gp"], ref["gp"]).max()
    print("per-launch vs persistent: u %.2e dp %.2e" % (du, dg), flush=True)
    assert du <= 1e-5 and dg <= 1e-4


def test_autotune_stores_and_reuses_its_choice():
    import torch

    import paper_2605_29155_amd as D
    d = W.make(3, B=256, T=50, seed=5004)
    dev = "cuda:0"
    h = handle()
    cfg = D.make_config(256, 50, 0, 3, 0.0, D.NEED_GRAD | D.TUNED)
    par = D.quad_params(W.quad_params_f32())
    t, o = _bufs(d, cfg, dev)
    assert D.get_tuned(h, cfg, True) is None
    # without a stored choice the flags decide (persistent, queue order)
    _run(D, h, cfg, par, t, o)
    assert D.last_launch_choice(h).plain == 0 and D.last_launch_choice(h).lpt == 0
    ch = D.autotune(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], t["T"], o["u"], o["x"], o["st"], o["ws"])
    torch.cuda.synchronize()
    tuned_u = o["u"].cpu().numpy().copy()
    print("autotune B=256 T=50: chose %s" % ch.as_dict(), flush=True)
    assert ch.ms > 0 and ch.waves_per_simd in (1, 2) and ch.grid_mode in (0, 1)
    got = D.get_tuned(h, cfg, True)
    assert got is not None and got.as_dict() == ch.as_dict()
    # another shape has no entry
    assert D.get_tuned(h, cfg, False) is None
    r = _run(D, h, cfg, par, t, o)
    used = D.last_launch_choice(h)
    assert (used.plain, used.lpt, used.waves_per_simd, used.grid_mode) == (ch.plain, ch.lpt, ch.waves_per_simd,
                                                                          ch.grid_mode)
    assert np.array_equal(r["u"], tuned_u)
    # the stored choice is validated
    with pytest.raises(D.DMPCError):
        D.set_tuned(h, cfg, True, D.LaunchChoice(0, 0, 3, 0, 0.0))


def test_layer_autotune_first_call_then_reuse():
    import torch

    import paper_2605_29155_amd as D
    d = W.make(1, B=128)
    dev = "cuda:0"
    layer = D.DMPCLayer(W.quad_params_f32(), max_iter=5, autotune=True)
    args = [torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi")]
    u1, _, _ = layer(*args)
    cfg = layer.config(128, d["T_max"], need_grad=False)
    got = D.get_tuned(layer.handle, cfg, False)
    assert got is not None
    u2, _, _ = layer(*args)
    used = D.last_launch_choice(layer.handle)
    assert (used.plain, used.waves_per_simd, used.grid_mode) == (got.plain, got.waves_per_simd, got.grid_mode)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
