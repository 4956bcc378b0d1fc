"""dmpc_forward_noalloc (the forward on the library's static device
workspace, for callers that cannot allocate) called through the C ABI gives
the outputs of dmpc_forward on a caller workspace, on two calls in a row, the
second smaller than the first, so the second runs on what the first left in
the shared array; sizes beyond the static array and DMPC_NEED_GRAD are
refused before anything is launched."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from gpu_util import handle, oracle_replay, parity_errors, within_bars, describe

pytestmark = pytest.mark.gpu


def _inputs(d, dev):
    import torch
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi")}
    t["T"] = torch.from_numpy(d["T"].astype(np.int32)).to(dev)
    return t


def _outputs(B, Tm, K, dev):
    import torch
    return dict(u=torch.full((B, Tm, 4), float("nan"), device=dev),
                x=torch.full((B, Tm, 13), float("nan"), device=dev),
                st=torch.full((B,), -1, dtype=torch.int32, device=dev),
                dl=torch.full((B, K, 1 + Tm), 77, dtype=torch.uint8, device=dev))


def _run_pair(d, flags):
    """Both entry points, raw C ABI, on the same inputs; returns numpy outputs."""
    import torch

    import paper_2605_29155_amd as D
    dev = "cuda:0"
    h = handle()
    L = D.lib()
    B, Tm, K = d["B"], d["T_max"], d["K"]
    cfg = D.make_config(B, Tm, d["cost_kind"], K, d["tol"], flags)
    par = D.quad_params(W.quad_params_f32())
    t = _inputs(d, dev)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    ptr = lambda a: None if a is None else C.c_void_p(a.data_ptr())  # noqa: E731
    ref = _outputs(B, Tm, K, dev)
    ws = D.alloc_workspace(cfg, dev)
    rc = L.dmpc_forward(h._h, C.byref(cfg), par, ptr(t["x0"]), ptr(t["Q"]), ptr(t["p"]), ptr(t["lo"]), ptr(t["hi"]),
                        ptr(t["T"]), None, ptr(ref["u"]), ptr(ref["x"]), ptr(ref["st"]), ptr(ws), ws.numel(),
                        ptr(ref["dl"]), s)
    assert rc == 0, L.dmpc_last_error(h._h)
    new = _outputs(B, Tm, K, dev)
    rc = L.dmpc_forward_noalloc(h._h, C.byref(cfg), par, ptr(t["x0"]), ptr(t["Q"]), ptr(t["p"]), ptr(t["lo"]),
                                ptr(t["hi"]), ptr(t["T"]), None, ptr(new["u"]), ptr(new["x"]), ptr(new["st"]),
                                ptr(new["dl"]), s)
    assert rc == 0, L.dmpc_last_error(h._h)
    torch.cuda.synchronize()
    cpu = lambda o: {k: v.cpu().numpy() for k, v in o.items()}  # noqa: E731
    return cpu(ref), cpu(new)


@pytest.mark.parametrize("flags_name", ["persistent-lpt", "per-launch"])
def test_noalloc_forward_equals_forward_twice(flags_name):
    import paper_2605_29155_amd as D
    flags = D.LPT if flags_name == "persistent-lpt" else D.PLAIN
    # first call: full-size metric-shaped forward (B = 1024, T = 20); second: a
    # smaller ragged batch with horizons 0, 1, 2 on the array the first left
    first = W.make(1)
    second = W.make(3, B=40, T=30, seed=4242)
    second["T"][:3] = [0, 1, 2]
    for d in (first, second):
        ref, new = _run_pair(d, flags)
        for k in ("u", "x", "st", "dl"):
            assert np.array_equal(ref[k], new[k]), (flags_name, d["B"], k)
        # and within the parity bars of the oracle replaying the decisions
        g = dict(u=new["u"], status=new["st"].astype(np.uint32), dlog=new["dl"], K=d["K"])
        idx = np.arange(min(d["B"], 64))
        o = oracle_replay(d, g, idx=idx, free=False)
        e = parity_errors(g, o, idx)
        print("noalloc %s B=%d T=%d: bitwise equal to dmpc_forward; %s"
              % (flags_name, d["B"], d["T_max"], describe(e)), flush=True)
        assert np.all(within_bars(e)), describe(e)


def test_noalloc_refusals():
    import torch

    import paper_2605_29155_amd as D
    h = handle()
    L = D.lib()
    par = D.quad_params(W.quad_params_f32())
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    dev = "cuda:0"
    x0 = torch.zeros(8, 13, device=dev)
    Q = torch.ones(8, 10, 17, device=dev)
    p = torch.zeros(8, 10, 17, device=dev)
    lo, hi = torch.zeros(8, 4, device=dev), torch.full((8, 4), 8.5, device=dev)
    u = torch.empty(8, 10, 4, device=dev)
    st = torch.empty(8, dtype=torch.int32, device=dev)
    ptr = lambda a: C.c_void_p(a.data_ptr())  # noqa: E731
    args = (ptr(x0), ptr(Q), ptr(p), ptr(lo), ptr(hi), None, None, ptr(u), None, ptr(st), None, s)
    # a backward would need the workspace: refused
    cfg = D.make_config(8, 10, 0, 5, 0.0, D.NEED_GRAD)
    assert L.dmpc_forward_noalloc(h._h, C.byref(cfg), par, *args) == -1
    # larger than the static array (B = 8192, T = 20 needs ~110 MB): refused, nothing launched
    big = D.make_config(8192, 20)
    assert D.workspace_bytes(big) > D.NOALLOC_WORKSPACE_BYTES
    assert L.dmpc_forward_noalloc(h._h, C.byref(big), par, *args) == -2
    assert b"static" in L.dmpc_last_error(h._h)
    assert h.launch_count() == 0
    # B = 0: nothing to do
    z = D.make_config(0, 10)
    assert L.dmpc_forward_noalloc(h._h, C.byref(z), par, *args) == 0
    torch.cuda.synchronize()
