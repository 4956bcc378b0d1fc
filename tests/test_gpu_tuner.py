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


@pytest.mark.parametrize("cfg_id", [3, 4], ids=["ragged-diag", "dense"])
def test_every_persistent_choice_is_bitwise_identical(cfg_id):
    import paper_2605_29155_amd as D
    d = W.make(cfg_id, B=96, T=20, seed=5003)
    dev = "cuda:0"
    h = handle()
    cfg = D.make_config(96, 20, d["cost_kind"], 4, 1e-5 if cfg_id == 3 else 0.0, D.NEED_GRAD | D.TUNED)
    par = D.quad_params(W.quad_params_f32())
    t, o = _bufs(d, cfg, dev)
    ref = None
    choices = [(occ, grid, lpt, 4) for occ in (1, 2) for grid in (0, 1) for lpt in (0, 1)]
    # fewer instances per wave (96 is not a multiple of 4 times either, so the
    # last unit is partly empty): the same bits
    choices += [(1, grid, lpt, ipw) for ipw in (2, 1) for grid in (0, 1) for lpt in (0, 1)]
    for occ, grid, lpt, ipw in choices:
        ch = D.LaunchChoice(0, lpt, occ, grid, 0.0, ipw)
        D.set_tuned(h, cfg, True, ch)
        r = _run(D, h, cfg, par, t, o)
        used = D.last_launch_choice(h)
        assert (used.plain, used.lpt, used.waves_per_simd, used.grid_mode, used.inst_per_wave) == \
            (0, lpt, occ, grid, ipw)
        if ref is None:
            ref = r
        for k in r:
            assert np.array_equal(r[k], ref[k]), (occ, grid, lpt, ipw, k)
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


def test_tuned_choices_saved_and_loaded(tmp_path):
    """Launch choices persist across handles through the tuning file, keyed by
    the device's architecture: a new handle that loads the file launches the
    stored choice; lines for another architecture, malformed lines and
    out-of-range choices are skipped."""
    import paper_2605_29155_amd as D
    h = handle()
    c1 = D.make_config(64, 12, 0, 3, 0.0, D.NEED_GRAD | D.TUNED)
    c2 = D.make_config(128, 30, 1, 5, 1e-5, D.TUNED, ckpt_every=10)
    c3 = D.make_config(32, 50, 0, 5, 0.0, D.TUNED)
    D.set_tuned(h, c1, True, D.LaunchChoice(0, 1, 2, 1, 0.5))
    D.set_tuned(h, c2, False, D.LaunchChoice(1, 0, 1, 0, 0.25))
    D.set_tuned(h, c3, False, D.LaunchChoice(0, 0, 1, 1, 0.125, 1))
    path = tmp_path / "tuned.txt"
    n = D.tuned_save(h, str(path))
    assert n >= 3
    lines = path.read_text().splitlines()
    assert len(lines) == n and all(s.startswith("dmpc-tuned-v1 gfx950") for s in lines)
    # another architecture, a malformed line and an out-of-range choice
    arch, cu = lines[0].split()[1:3]
    extra = ["dmpc-tuned-v1 gfx942 %s 64 12 0 1 0 1 0 0 2 0 0.1" % cu, "dmpc-tuned-v1 %s %s 1 2" % (arch, cu),
             "dmpc-tuned-v1 %s %s 9 9 0 0 0 0 0 0 7 0 0.1" % (arch, cu)]
    path.write_text("\n".join(lines + extra) + "\n")
    h2 = D.Handle(0)
    assert D.get_tuned(h2, c1, True) is None
    assert D.tuned_load(h2, str(path)) == n
    g1, g2 = D.get_tuned(h2, c1, True), D.get_tuned(h2, c2, False)
    assert g1.as_dict() == dict(plain=0, lpt=1, waves_per_simd=2, grid_mode=1, ms=0.5, inst_per_wave=4)
    assert g2.as_dict() == dict(plain=1, lpt=0, waves_per_simd=1, grid_mode=0, ms=0.25, inst_per_wave=4)
    assert D.get_tuned(h2, c3, False).inst_per_wave == 1
    assert D.get_tuned(h2, D.make_config(9, 9), False) is None
    # a line without the instances-per-wave field (the earlier format) reads as 4
    old = [ln for ln in lines if ln.split()[3:9] == ["64", "12", "0", "1", "0", "1"]][0]
    path.write_text(" ".join(old.split()[:-1]) + "\n")
    h3 = D.Handle(0)
    assert D.tuned_load(h3, str(path)) == 1 and D.get_tuned(h3, c1, True).inst_per_wave == 4
    with pytest.raises(D.DMPCError):
        D.tuned_load(h2, str(tmp_path / "missing.txt"))


def test_layer_tune_file_round_trip(tmp_path):
    """A layer with a tune_file tunes a new shape once and writes the file; a
    second layer built on that file starts with the choice and does not tune
    again; both give the same solution."""
    import torch

    import paper_2605_29155_amd as D
    d = W.make(1, B=64, T=12, seed=5100)
    dev = "cuda:0"
    path = str(tmp_path / "tuned.txt")
    args = [torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi")]
    l1 = D.DMPCLayer(W.quad_params_f32(), max_iter=3, autotune=True, tune_file=path)
    u1, _, _ = l1(*args)
    cfg = l1.config(64, 12, need_grad=False)
    c1 = D.get_tuned(l1.handle, cfg, False)
    assert c1 is not None and (tmp_path / "tuned.txt").exists()
    l2 = D.DMPCLayer(W.quad_params_f32(), max_iter=3, autotune=True, tune_file=path)
    c2 = D.get_tuned(l2.handle, cfg, False)
    assert c2 is not None and c2.as_dict() == c1.as_dict()
    u2, _, _ = l2(*args)
    torch.cuda.synchronize()
    assert torch.equal(u1, u2)
