"""Helpers for the GPU parity tests: run the HIP library through its C ABI and
compare with the FP64 oracle, which replays the kernel's discrete decisions
(line-search choice, box-QP clamp patterns, iteration count, final active
set) so that the comparison isolates arithmetic from decisions."""
import numpy as np

import oracle as orc
import workloads as W

_handle = None


def handle():
    global _handle
    import paper_2605_29155_amd as D
    if _handle is None:
        _handle = D.Handle(0)
    return _handle


def rel(a, b, axis_from=1):
    """Per-instance normwise relative error ||a - b||_2 / max(||b||_2, 1e-6)."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1e-6)


def maxabs(a, b):
    """Per-instance element-wise error max_i |a_i - b_i| / max(1, max_i |b_i|)."""
    a = np.asarray(a, np.float64).reshape(a.shape[0], -1)
    b = np.asarray(b, np.float64).reshape(b.shape[0], -1)
    return np.abs(a - b).max(axis=1) / np.maximum(1.0, np.abs(b).max(axis=1))


def replay_violation(o):
    """Per-instance worst score of the kernel's clamp patterns, replayed by the
    oracle, against the oracle's own stage QPs (Sec. IV, backward pass with
    input bounds): 0 when every replayed pattern satisfies the QP's optimality
    conditions (free controls inside the box, clamped ones with correctly
    signed multipliers), else the smallest relative tolerance at which all do."""
    v = o["replay"]["replay_viol"]
    return v.reshape(v.shape[0], -1).max(axis=1)


# bars of the parity tests: 1e-4 relative on u*, 1e-3 on the gradients, both
# normwise per instance and element-wise (max-abs over max(1, max |ref|));
# the replayed clamp patterns must satisfy the oracle's stage QPs to 1e-4
TOL_U, TOL_G, TOL_VIOL = 1e-4, 1e-3, 1e-4
GRADS = ("dQ", "dp", "dx0")


def parity_errors(g, o, idx=None):
    """Per-instance errors of the kernel's outputs g (rows idx) against the
    oracle o that replayed its decisions on those rows: u (normwise), u_abs
    (element-wise), g and g_abs (worst of dQ, dp, dx0), viol (replayed
    patterns against the oracle's stage QPs)."""
    sel = slice(None) if idx is None else idx
    e = dict(u=rel(g["u"][sel], o["replay"]["u"]), u_abs=maxabs(g["u"][sel], o["replay"]["u"]),
             viol=replay_violation(o))
    if "bwd" in o and "dQ" in g:
        e["g"] = np.max([rel(g[k][sel], o["bwd"][k]) for k in GRADS], axis=0)
        e["g_abs"] = np.max([maxabs(g[k][sel], o["bwd"][k]) for k in GRADS], axis=0)
    return e


def within_bars(e, scale=1.0):
    """Per-instance: every error of parity_errors within its bar (times scale)."""
    ok = (e["u"] <= TOL_U * scale) & (e["u_abs"] <= TOL_U * scale) & (e["viol"] <= TOL_VIOL * scale)
    if "g" in e:
        ok &= (e["g"] <= TOL_G * scale) & (e["g_abs"] <= TOL_G * scale)
    return ok


def describe(e):
    s = "u* %.2e (abs %.2e)" % (e["u"].max(), e["u_abs"].max())
    if "g" in e:
        s += " | grads %.2e (abs %.2e)" % (e["g"].max(), e["g_abs"].max())
    return s + " | pattern violation %.1e" % e["viol"].max()


def run_gpu(d, plain=False, lpt=True, need_grad=True, K=None, tol=None, dlog=True, grad_u=None, grad_x=None,
            fp64_pivot=1e-6, ckpt=0, theta=False, tpar=False, f64=False, redo=False, tuned=False):
    import torch

    import paper_2605_29155_amd as D
    dev = "cuda:0"
    h = handle()
    B, Tm = d["B"], d["T_max"]
    K = d["K"] if K is None else K
    tol = d["tol"] if tol is None else tol
    flags = (D.NEED_GRAD if need_grad else 0) | (D.PLAIN if plain else 0) | (D.LPT if lpt else 0)
    flags |= D.TPAR if tpar else 0
    flags |= D.F64 if f64 else 0
    flags |= D.F64_REDO if redo else 0
    flags |= D.TUNED if tuned else 0
    cfg = D.make_config(B, Tm, d["cost_kind"], K, tol, flags, fp64_pivot, ckpt)
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi")}
    Tt = torch.from_numpy(d["T"].astype(np.int32)).to(dev)
    ws = D.alloc_workspace(cfg, dev)
    u = torch.full((B, Tm, 4), float("nan"), device=dev)
    x = torch.full((B, Tm, 13), float("nan"), device=dev)
    st = torch.zeros(B, dtype=torch.int32, device=dev)
    dl = torch.zeros((B, max(K, 1), 1 + Tm), dtype=torch.uint8, device=dev) if dlog else None
    par = D.quad_params(W.quad_params_f32())
    if tuned:
        # the launch choice the autotuner keeps for this shape (as the bench runs it)
        D.autotune(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], Tt, u, x, st, ws)
    D.forward_raw(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], Tt, u, x, st, ws, dl)
    out = dict(launches_fwd=h.launch_count())
    if need_grad:
        gu = torch.from_numpy(np.ascontiguousarray(d["grad_u"] if grad_u is None else grad_u)).to(dev)
        gx = None if grad_x is None else torch.from_numpy(np.ascontiguousarray(grad_x)).to(dev)
        gQ = torch.full_like(t["Q"], float("nan"))
        gp = torch.full_like(t["p"], float("nan"))
        gx0 = torch.full_like(t["x0"], float("nan"))
        gd = torch.full((B, 8), float("nan"), device=dev) if theta else None
        D.backward_raw(h, cfg, par, t["Q"], t["p"], t["lo"], t["hi"], ws, gu, gx, gQ, gp, gx0, grad_dyn=gd)
        out["launches_bwd"] = h.launch_count()
    torch.cuda.synchronize()
    out.update(u=u.cpu().numpy(), x=x.cpu().numpy(), status=st.cpu().numpy().astype(np.uint32), K=K)
    if dlog:
        out["dlog"] = dl.cpu().numpy()
    if need_grad:
        out.update(dQ=gQ.cpu().numpy(), dp=gp.cpu().numpy(), dx0=gx0.cpu().numpy())
        if theta:
            out["gdyn"] = gd.cpu().numpy()
    return out


def oracle_replay(d, g, idx=None, grad_u=None, grad_x=None, free=True):
    """FP64 oracle on the same inputs, replaying the kernel's decisions; also
    (free=True) a free oracle run for the decision-agreement rate."""
    P = orc.params_from(W.quad_params_f32())
    sel = slice(None) if idx is None else idx
    x0, Q, p, lo, hi, T = (np.asarray(d[k])[sel] for k in ("x0", "Q", "p", "lo", "hi", "T"))
    gu = np.asarray(d["grad_u"] if grad_u is None else grad_u)[sel]
    gx = None if grad_x is None else np.asarray(grad_x)[sel]
    K = g["K"]
    iters = ((g["status"][sel] >> 8) & 255).astype(np.int32)
    dl = g["dlog"][sel]
    alpha, pattern = dl[:, :K, 0], dl[:, :K, 1:]
    fr = orc.forward(P, x0, Q, p, lo, hi, T, K=K, replay=(iters, alpha, pattern))
    ff = orc.forward(P, x0, Q, p, lo, hi, T, K=K, tol=d["tol"]) if free else None
    out = dict(replay=fr, free=ff, iters=iters, alpha=alpha, pattern=pattern)
    if "dQ" in g:
        mask = orc.active_mask(g["u"][sel], lo, hi, T)
        out["bwd"] = orc.backward(P, x0, Q, p, lo, hi, fr["u"], fr["x"], gu, gx, T=T, mask=mask,
                                  dtheta="gdyn" in g)
    return out


def decision_agreement(g, o, idx=None):
    """Fraction of instances whose free-run oracle decisions (alpha per
    iteration, box-QP patterns, iteration count) equal the kernel's."""
    sel = slice(None) if idx is None else idx
    ff = o["free"]
    K = g["K"]
    same = np.ones(len(o["iters"]), bool)
    same &= ff["iters"] == o["iters"]
    for b in range(len(same)):
        k = o["iters"][b]
        same[b] &= np.array_equal(ff["alpha"][b, :k], o["alpha"][b, :k])
        same[b] &= np.array_equal(ff["pattern"][b, :k], o["pattern"][b, :k])
    return same.mean()


def pattern_agreement(o):
    """Fraction of instances whose free-run oracle takes the kernel's box-QP
    clamp patterns at every stage of every iteration it ran and the same
    number of iterations (the line-search choices left out: where the
    candidates' costs tie to rounding, e.g. once the steps have become tiny,
    the first minimiser is decided by rounding alone; alpha_choices_valid
    checks those choices)."""
    ff = o["free"]
    same = ff["iters"] == o["iters"]
    for b in range(len(same)):
        k = o["iters"][b]
        same[b] &= np.array_equal(ff["pattern"][b, :k], o["pattern"][b, :k])
    return same.mean()


def alpha_choices_valid(o, rtol=1e-4):
    """Every kernel line-search choice is a minimiser of the oracle's candidate
    costs up to rounding (the choice is a floating-point decision)."""
    cc = o["replay"]["cand_cost"]
    bad = 0
    for b in range(cc.shape[0]):
        for k in range(o["iters"][b]):
            a = o["alpha"][b, k]
            if a == 255:
                continue
            m = np.min(cc[b, k])
            if cc[b, k, a] > m + rtol * (1 + abs(m)):
                bad += 1
    return bad


def oracle_sensitivity(d, o, idx=None, orows=None, trials=3, eps=1e-7, seed=0):
    """Conditioning of each instance's solution map at FP32 resolution: the
    largest normwise change of the FP64 oracle's u* (decisions replayed from
    the kernel) when Q, p and x0 get independent relative perturbations of
    size eps (about one FP32 rounding).  A kernel that rounds to FP32 at every
    stage of every iteration cannot agree with the oracle much better than
    this on an instance where it is large.  idx: rows of d; orows: the rows
    of o that belong to them (default all of o)."""
    P = orc.params_from(W.quad_params_f32())
    sel = slice(None) if idx is None else idx
    x0, Q, p, lo, hi, T = (np.asarray(d[k])[sel].astype(np.float64) for k in ("x0", "Q", "p", "lo", "hi", "T"))
    T = T.astype(np.int32)
    osel = slice(None) if orows is None else orows
    rep = (o["iters"][osel], o["alpha"][osel], o["pattern"][osel])
    K = o["alpha"].shape[1]
    base = o["replay"]["u"][osel]
    rng = np.random.default_rng(seed)
    s = np.zeros(len(base))
    for _ in range(trials):
        pert = [a * (1 + eps * rng.standard_normal(a.shape)) for a in (x0, Q, p)]
        f = orc.forward(P, pert[0], pert[1], pert[2], lo, hi, T, K=K, replay=rep)
        s = np.maximum(s, rel(f["u"], base))
    return s
