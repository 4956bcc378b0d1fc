"""Benchmark of the batched differentiable MPC layer (forward + backward).

Workload: batch 4096, horizon 20, 5 iLQR iterations, 13-state quadrotor,
diagonal stage cost emitted per instance by a random-init 2x256 tanh MLP
(synthetic inputs; the MLP runs once before timing and is not timed).  A step
is one forward solve plus one backward of the whole batch, replayed from a HIP
graph of the persistent form; the per-launch form (init, three launches per
iteration, tail, outputs, backward) is timed beside it on the same inputs.

Prints one JSON line.  The CPU baseline leg times the FP64 oracle on the host
cores and checks the kernel's results against it on a sample (decisions
replayed).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# canonical FLOP model per stage (1 FMA = 2 FLOP), diagonal / dense cost:
# RK4 + nominal linearisation by the chain rule, cost gradient, Riccati with
# box-QP, four-candidate line search; forward tail (linearise + fixed-mask
# Riccati at the solution); adjoint sweeps; initial rollout.
FLOP = dict(iter_stage=(27416, 30204), tail=(23478, 23478), adjoint=(1200, 2500), init=(593, 593))
# MI355X published vector peaks: FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s (bench.py --peaks measures 139 and
# 75 with single FMAs, no packed FP32).  The headline fraction is against the FP32 peak; the fraction
# against the FP64 peak is reported beside it, since a quarter of the forward's VALU instructions are FP64
# FMAs.
PEAK_FP32 = 157.3e12
PEAK_FP64 = 78.6e12
HBM_PEAK = 8.0e12


def flops_per_solve(T, K, dense=False):
    i = 1 if dense else 0
    fwd = T * (FLOP["init"][i] + K * FLOP["iter_stage"][i] + FLOP["tail"][i])
    return fwd, T * FLOP["adjoint"][i]


def kernel_source_hash():
    """Hash of the kernel sources and the compiler flags they are built with."""
    from paper_2605_29155_amd import build as _b
    h = hashlib.sha256()
    for f in ("paper_2605_29155_amd/csrc/dmpc.hip", "paper_2605_29155_amd/csrc/dmpc_device.hpp",
              "paper_2605_29155_amd/csrc/dmpc_theta.hpp", "include/dmpc.h"):
        h.update(open(os.path.join(ROOT, f), "rb").read())
    h.update(" ".join(f for f in _b.FLAGS if not f.startswith("-I")).encode())
    return h.hexdigest()[:16]


def load_traffic(kernel_hash, B):
    """HBM bytes per launch of the persistent forward kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary, if taken on this kernel source."""
    p = os.path.join(ROOT, "profiles", "traffic_fwd_persistent_b4096_t20.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_source_hash") != kernel_hash or d.get("B") != B:
        return None
    return d.get("hbm_bytes_per_launch")


def make_inputs(dev, B=None):
    import numpy as np
    import torch

    import workloads as W
    d = W.make(2) if B is None else W.make(2, B=B)
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi", "grad_u")}
    t["T"] = torch.from_numpy(d["T"]).to(dev)
    return d, t


def event_times(run, s, n):
    """HIP-event time (ms) of each of n calls of run() on stream s."""
    import torch
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for e0, e1 in ev:
        e0.record(s)
        run()
        e1.record(s)
    s.synchronize()
    return [e0.elapsed_time(e1) for e0, e1 in ev]


def pct(v):
    """median, p10, p90 of a list of times."""
    import numpy as np
    v = np.asarray(v, np.float64)
    return dict(median=float(np.median(v)), p10=float(np.percentile(v, 10)), p90=float(np.percentile(v, 90)), n=len(v))


def run_gpu_bench(d, t, steps, warmup, replays=100):
    """Times the fwd+bwd step of the tuned persistent form (captured in a HIP
    graph: the headline) and of the per-launch form (eager, and captured in a
    graph too), all on the same inputs.  Per form: wall-clock mean over
    `steps` steps after `warmup` (the headline's timed region), HIP-event
    median / p10 / p90 over `replays` single steps, the forward call's own
    HIP-event time, and the outputs of the last step."""
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = t["x0"].device
    B, Tm, K = d["B"], d["T_max"], d["K"]
    h = D.Handle(0)
    params = D.quad_params(W.quad_params_f32())
    out = {}
    for form in ("persistent", "plain", "fp64"):
        # the headline form uses the launch the autotuner picks for this shape;
        # "fp64" is the FP64 form (DMPC_F64), tuned the same way
        flags = D.NEED_GRAD | (D.PLAIN if form == "plain" else D.LPT | D.TUNED)
        flags |= D.F64 if form == "fp64" else 0
        cfg = D.make_config(B, Tm, D.COST_DIAG, K, 0.0, flags)
        ws = D.alloc_workspace(cfg, dev)
        u = torch.empty(B, Tm, 4, device=dev)
        x = torch.empty(B, Tm, 13, device=dev)
        st = torch.empty(B, dtype=torch.int32, device=dev)
        gQ, gp, gx0 = torch.empty_like(t["Q"]), torch.empty_like(t["p"]), torch.empty_like(t["x0"])
        s = torch.cuda.Stream()

        def fwd():
            D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws, None, s)

        def step():
            fwd()
            D.backward_raw(h, cfg, params, None, None, None, None, ws, t["grad_u"], None, gQ, gp, gx0, s)

        choice = None
        if form != "plain":
            with torch.cuda.stream(s):
                choice = D.autotune(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws,
                                    s).as_dict()
        with torch.cuda.stream(s):
            step()
        torch.cuda.synchronize()
        fwd()
        launches = h.launch_count() + 1
        # graph of the whole fwd+bwd step
        D.capture_begin(h, s)
        step()
        g = D.capture_end(h, s)
        graph = lambda: D.graph_launch(h, g, s)  # noqa: E731
        timed = graph if form != "plain" else step
        for _ in range(warmup):
            timed()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            timed()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        for _ in range(10):
            graph()
        ev_graph = pct(event_times(graph, s, replays))
        for _ in range(10):
            step()
        ev_eager = pct(event_times(step, s, replays))
        # dominant kernel: the forward call (queue reset + the forward kernel in
        # the persistent form), HIP events on the stream it is launched on
        ev_fwd = pct(event_times(fwd, s, 20))
        graph()
        torch.cuda.synchronize()
        out[form] = dict(s_per_step=dt, graph_step_ms=ev_graph, eager_step_ms=ev_eager, fwd_ms=ev_fwd["median"],
                         fwd_ms_events=ev_fwd, launches=launches, choice=choice,
                         u=u.cpu().numpy(), x=x.cpu().numpy(), status=st.cpu().numpy().astype("uint32"),
                         dQ=gQ.cpu().numpy(), dp=gp.cpu().numpy(), dx0=gx0.cpu().numpy())
        D.graph_destroy(h, g)
    return out


def torch_steps(d, t, steps=20, warmup=3):
    """The layer as a torch module user calls it: DMPCLayer (the module-level
    autograd.Function, autotuned) on the same inputs, loss sum_b u*_b,0 . w_b,
    loss.backward().  layer_ms: x0, Q, p given as leaf tensors; full_ms: the
    cost MLP on the GPU emits Q, p (forward and backward through it too).
    Wall-clock mean per step, stream synchronised."""
    import numpy as np
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = t["x0"].device
    layer = D.DMPCLayer(W.quad_params_f32(), max_iter=d["K"], autotune=True)
    w = torch.from_numpy(d["w"]).to(dev)
    x0 = t["x0"].clone().requires_grad_(True)
    Q = t["Q"].clone().requires_grad_(True)
    p = t["p"].clone().requires_grad_(True)
    mlp = W.CostMLP(d["T_max"], W.CONFIGS[2]["seed"], device=dev)
    inp = torch.from_numpy(np.ascontiguousarray(d["mlp_input"])).to(dev)

    def layer_step():
        for a in (x0, Q, p):
            a.grad = None
        u, _, _ = layer(x0, Q, p, t["lo"], t["hi"])
        (u[:, 0, :] * w).sum().backward()

    def full_step():
        for a in mlp.params:
            a.grad = None
        Qm, pm = mlp(inp)
        u, _, _ = layer(t["x0"], Qm, pm, t["lo"], t["hi"])
        (u[:, 0, :] * w).sum().backward()

    res = {}
    for name, fn in (("layer_ms", layer_step), ("full_ms", full_step)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps * 1e3
    # the layer's gradients equal the raw C ABI's on the same inputs
    layer_step()
    res["dp_layer"] = p.grad.cpu().numpy()
    return res


def profile_short(d, t):
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = t["x0"].device
    B, Tm, K = d["B"], d["T_max"], d["K"]
    h = D.Handle(0)
    cfg = D.make_config(B, Tm, D.COST_DIAG, K, 0.0, D.NEED_GRAD | D.LPT)
    ws = D.alloc_workspace(cfg, dev)
    u = torch.empty(B, Tm, 4, device=dev)
    x = torch.empty(B, Tm, 13, device=dev)
    st = torch.empty(B, dtype=torch.int32, device=dev)
    gQ, gp, gx0 = torch.empty_like(t["Q"]), torch.empty_like(t["p"]), torch.empty_like(t["x0"])
    params = D.quad_params(W.quad_params_f32())
    for _ in range(2):
        D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws)
        D.backward_raw(h, cfg, params, None, None, None, None, ws, t["grad_u"], None, gQ, gp, gx0)
    torch.cuda.synchronize()
    n = 256 << 20
    src = torch.ones(n // 4, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print("profile-short: 2 x (fwd + bwd), then a %d-byte device copy" % n, flush=True)


# Table I of the paper (solver latency, drone hover at random targets; RTX A6000 + i9-13900K):
# (B, T) -> (CA-DiffMPC forward ms, CA-DiffMPC backward ms)
PAPER_TABLE1 = {(1, 2): (0.93, 0.32), (1, 10): (1.08, 0.80), (1, 50): (1.84, 2.35),
                (256, 2): (1.21, 0.38), (256, 10): (1.68, 0.87), (256, 50): (4.00, 2.60)}


def latency_table(reps=20, warmup=3):
    """Forward and backward latency of one call (HIP events on the call's
    stream, median of `reps`) at the paper's latency shapes, hover-to-target
    workload, K = 5 (the paper does not state K for this table)."""
    import numpy as np
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = "cuda:0"
    h = D.Handle(0)
    params = D.quad_params(W.quad_params_f32())
    rows = []
    for (B, T), (pf, pb) in PAPER_TABLE1.items():
        d = W.make_hover_target(B, T)
        t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi", "grad_u")}
        cfg = D.make_config(B, T, D.COST_DIAG, d["K"], 0.0, D.NEED_GRAD)
        ws = D.alloc_workspace(cfg, dev)
        u = torch.empty(B, T, 4, device=dev)
        x = torch.empty(B, T, 13, device=dev)
        st = torch.empty(B, dtype=torch.int32, device=dev)
        gQ, gp, gx0 = torch.empty_like(t["Q"]), torch.empty_like(t["p"]), torch.empty_like(t["x0"])
        s = torch.cuda.Stream()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        fw, bw = [], []
        with torch.cuda.stream(s):
            for r in range(warmup + reps):
                e[0].record(s)
                D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws, None, s)
                e[1].record(s)
                D.backward_raw(h, cfg, params, None, None, None, None, ws, t["grad_u"], None, gQ, gp, gx0, s)
                e[2].record(s)
                e[2].synchronize()
                if r >= warmup:
                    fw.append(e[0].elapsed_time(e[1]))
                    bw.append(e[1].elapsed_time(e[2]))
        f, b = float(np.median(fw)), float(np.median(bw))
        rows.append(dict(B=B, T=T, K=d["K"], fwd_ms=f, bwd_ms=b, solves_per_s=B / ((f + b) * 1e-3),
                         paper_fwd_ms=pf, paper_bwd_ms=pb, status_converged=None))
        print("latency B=%3d T=%2d: fwd %.3f ms (paper %.2f)  bwd %.3f ms (paper %.2f)" % (B, T, f, pf, b, pb),
              file=sys.stderr, flush=True)
    return rows


def closed_loop_latency(steps=40, warmup=5):
    """Latency of one receding-horizon control step at B = 1 (forward solve
    from the current state + apply u*_0 + shift), hover-to-target workload,
    for T 10, 20, 50: fixed K = 5, and K <= 30 stopping at ||dU||_inf < 1e-5,
    each cold (every solve from hover thrust) and warm (from the shifted
    previous solution), the warm loop also as one captured HIP graph per step
    and, warm, with the per-launch form whose backward pass is the
    time-parallel Riccati (DMPC_TPAR).
    wall_ms: host time from the call to the step's completion (stream
    synchronised); gpu_ms: HIP events around the step on its stream.  Each
    variant runs twice, in the order cold, warm, graph and then reversed (so
    that clock ramps do not favour one), `steps` timed steps of a running
    closed loop after `warmup` steps each time; medians over both runs."""
    import numpy as np
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    from paper_2605_29155_amd.receding import RecedingHorizon
    dev = "cuda:0"
    h = D.Handle(0)

    def run(t, T, K, tol, warm, graph, tpar=False):
        rh = RecedingHorizon(W.quad_params_f32(), 1, T, max_iter=K, tol_du=tol, warm=warm, handle=h, tpar=tpar)
        rh.reset(t["x0"])
        s = torch.cuda.Stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        wall, gpu, its = [], [], []
        with torch.cuda.stream(s):
            if graph:
                rh.step(t["Q"], t["p"], t["lo"], t["hi"], stream=s)
                s.synchronize()
                rh.capture(t["Q"], t["p"], t["lo"], t["hi"], stream=s)
            for r in range(warmup + steps):
                s.synchronize()
                c0 = time.perf_counter()
                e0.record(s)
                if graph:
                    rh.replay()
                else:
                    rh.step(t["Q"], t["p"], t["lo"], t["hi"], stream=s)
                e1.record(s)
                s.synchronize()
                c1 = time.perf_counter()
                if r >= warmup:
                    wall.append((c1 - c0) * 1e3)
                    gpu.append(e0.elapsed_time(e1))
                    its.append((int(rh.status.item()) >> 8) & 255)
        rh.release()
        return wall, gpu, its, rh.x[0, :3].cpu().numpy()

    rows = []
    variants = ((False, False, False), (True, False, False), (True, True, False), (True, False, True),
                (True, True, True))
    for T in (10, 20, 50):
        d = W.make_hover_target(1, T)
        t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi")}
        target = -d["p"][0, 0, :3] / d["Q"][0, 0, :3]
        for K, tol in ((5, 0.0), (30, 1e-5)):
            acc = {v: ([], [], [], None) for v in variants}
            for v in variants + variants[::-1]:
                w, g, i, pos = run(t, T, K, tol, *v)
                acc[v] = (acc[v][0] + w, acc[v][1] + g, acc[v][2] + i, pos)
            for (warm, graph, tpar) in variants:
                w, g, i, pos = acc[(warm, graph, tpar)]
                row = dict(B=1, T=T, K=K, tol_du=tol, warm=warm, graph=graph, form="tpar" if tpar else "persistent",
                           wall_ms=float(np.median(w)),
                           wall_ms_p90=float(np.percentile(w, 90)), gpu_ms=float(np.median(g)),
                           mean_iters=float(np.mean(i)), median_iters=float(np.median(i)),
                           final_pos_err_m=float(np.linalg.norm(pos - target)))
                rows.append(row)
                print("closed loop T=%2d K=%2d tol=%g %-16s: wall %.3f ms (p90 %.3f), gpu %.3f ms, iterations "
                      "mean %.1f median %.0f" % (T, K, tol, ("warm" if warm else "cold") + ("+graph" if graph else "")
                                                 + ("+tpar" if tpar else ""),
                                                 row["wall_ms"], row["wall_ms_p90"], row["gpu_ms"],
                                                 row["mean_iters"], row["median_iters"]), file=sys.stderr, flush=True)
    return rows


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_leg(d, gpu, nsample=64):
    """The FP64 oracle on the host (never tuned; test infrastructure):
    - forward + Riccati-adjoint backward of the full batch on the host threads
      this process may use (at most 16), repeated for about 10 s;
    - the same on one thread, on the first 256 instances, scaled to solves/s;
    - the dense-KKT backward (the verification path) on 256 instances with
      all threads, its time per solve scaled linearly to the batch;
    and checks the kernel on a sample with its decisions replayed (one extra
    kernel run with the decision log): errors, decision agreement with a free
    oracle run, the fraction of controls on a bound, the iteration counts."""
    import numpy as np
    import torch

    import oracle as orc
    import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import (alpha_choices_valid, decision_agreement, maxabs, oracle_replay, pattern_agreement, rel,
                          replay_violation, run_gpu)
    P = orc.params_from(W.quad_params_f32())
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nthreads = max(1, min(16, avail))

    def fwd_bwd(sl, nt):
        a = {k: d[k][sl] for k in ("x0", "Q", "p", "lo", "hi", "T", "grad_u")}
        f = orc.forward(P, a["x0"], a["Q"], a["p"], a["lo"], a["hi"], a["T"], K=d["K"], nthreads=nt)
        orc.backward(P, a["x0"], a["Q"], a["p"], a["lo"], a["hi"], f["u"], f["x"], a["grad_u"], T=a["T"],
                     nthreads=nt)
        return f

    def repeat(fn, budget):
        t0, reps = time.perf_counter(), 0
        while True:
            fn()
            reps += 1
            wall = time.perf_counter() - t0
            if wall >= budget or reps >= 60:
                return reps, wall

    full = slice(None)
    reps, wall = repeat(lambda: fwd_bwd(full, nthreads), 10.0)
    n1 = min(256, d["B"])
    reps1, wall1 = repeat(lambda: fwd_bwd(slice(0, n1), 1), 3.0)
    f = fwd_bwd(slice(0, n1), nthreads)
    a = {k: d[k][:n1] for k in ("x0", "Q", "p", "lo", "hi", "T", "grad_u")}
    t0 = time.perf_counter()
    orc.backward(P, a["x0"], a["Q"], a["p"], a["lo"], a["hi"], f["u"], f["x"], a["grad_u"], T=a["T"], method=1,
                 nthreads=nthreads)
    kkt_s = time.perf_counter() - t0
    cpu = dict(value=reps * d["B"] / wall, unit="solves/s", cores=nthreads, kind="oracle",
               sample="full batch B=%d T=%d K=%d repeated %d times, FP64 forward + Riccati-adjoint backward, "
                      "%d threads, %.1f s wall" % (d["B"], d["T_max"], d["K"], reps, nthreads, wall),
               host_cpu=cpu_model(), host_nproc=os.cpu_count(), threads_available=avail,
               single_thread=dict(value=reps1 * n1 / wall1, unit="solves/s",
                                  sample="first %d instances repeated %d times on 1 thread, %.1f s wall"
                                         % (n1, reps1, wall1)),
               dense_kkt_backward=dict(ms_per_solve=kkt_s / n1 * 1e3, batch_s_scaled=kkt_s / n1 * d["B"],
                                       sample="%d instances, %d threads, %.2f s wall; scaled linearly to B=%d "
                                              "(instances are independent)" % (n1, nthreads, kkt_s, d["B"])))
    # accuracy on a sample, decisions replayed
    idx = np.arange(0, d["B"], d["B"] // nsample)[:nsample]
    g = run_gpu(d, lpt=True)
    o = oracle_replay(d, g, idx=idx)
    sel = lambda v: v[idx]  # noqa: E731
    acc = dict(sample=len(idx),
               u_rel_max=float(rel(sel(g["u"]), o["replay"]["u"]).max()),
               u_abs_max=float(maxabs(sel(g["u"]), o["replay"]["u"]).max()),
               dQ_rel_max=float(rel(sel(g["dQ"]), o["bwd"]["dQ"]).max()),
               dp_rel_max=float(rel(sel(g["dp"]), o["bwd"]["dp"]).max()),
               dx0_rel_max=float(rel(sel(g["dx0"]), o["bwd"]["dx0"]).max()),
               grad_abs_max=float(max(maxabs(sel(g[k]), o["bwd"][k]).max() for k in ("dQ", "dp", "dx0"))),
               replayed_pattern_violation_max=float(replay_violation(o).max()),
               decision_agreement=float(decision_agreement(g, o, idx)),
               pattern_agreement=float(pattern_agreement(o)),
               alpha_choices_not_a_minimiser=int(alpha_choices_valid(o)),
               decision_note="decision_agreement: every decision (step length, clamp patterns, iteration count) "
                             "equal to a free FP64 oracle run's; pattern_agreement leaves out the step lengths, "
                             "which tie to rounding once the steps are tiny; alpha_choices_not_a_minimiser counts "
                             "kernel step lengths whose oracle cost is not within 1e-4 of the minimum")
    # the timed persistent run and the decision-logged run must agree exactly
    acc["bench_run_matches_logged_run"] = bool(np.array_equal(gpu["persistent"]["u"], g["u"]))
    u = gpu["persistent"]["u"]
    lo, hi = d["lo"][:, None, :], d["hi"][:, None, :]
    acc["active_fraction"] = float(np.mean((u <= lo) | (u >= hi)))
    its = (gpu["persistent"]["status"] >> 8) & 255
    acc["iterations_histogram"] = {int(k): int(v) for k, v in zip(*np.unique(its, return_counts=True))}
    torch.cuda.synchronize()
    return cpu, acc


def _tensors(d, dev):
    import numpy as np
    import torch
    t = {k: torch.from_numpy(np.ascontiguousarray(d[k])).to(dev) for k in ("x0", "Q", "p", "lo", "hi", "grad_u")}
    t["T"] = torch.from_numpy(d["T"].astype(np.int32)).to(dev)
    return t


def _solver(h, d, t, flags, dev):
    """fwd / step closures of one launch form on workload d (horizons given)."""
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    B, Tm = d["B"], d["T_max"]
    cfg = D.make_config(B, Tm, d["cost_kind"], d["K"], d["tol"], flags, 1e-6, d["ckpt"])
    ws = D.alloc_workspace(cfg, dev)
    par = D.quad_params(W.quad_params_f32())
    o = dict(u=torch.empty(B, Tm, 4, device=dev), x=torch.empty(B, Tm, 13, device=dev),
             st=torch.empty(B, dtype=torch.int32, device=dev), gQ=torch.empty_like(t["Q"]),
             gp=torch.empty_like(t["p"]), gx0=torch.empty_like(t["x0"]))
    s = torch.cuda.Stream()

    def fwd():
        D.forward_raw(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], t["T"], o["u"], o["x"], o["st"], ws,
                      None, s)

    def step():
        fwd()
        D.backward_raw(h, cfg, par, t["Q"], t["p"], t["lo"], t["hi"], ws, t["grad_u"], None, o["gQ"], o["gp"],
                       o["gx0"], s)

    def tune():
        with torch.cuda.stream(s):
            return D.autotune(h, cfg, par, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], t["T"], o["u"], o["x"],
                              o["st"], ws, s).as_dict()

    return dict(cfg=cfg, ws=ws, out=o, s=s, fwd=fwd, step=step, tune=tune)


def config_lines(replays=20):
    """fwd+bwd step of the ragged workload (B=8192, T in 10..50, up to 10
    iterations with the ||du||_inf < 1e-5 stop, bounds hi ~ U[6,10]) and of
    the large dense one (B=16384, T=50, dense Wishart cost, checkpoints every
    10 stages): the autotuned persistent form and the per-launch form, each
    eager and captured in a HIP graph; HIP-event median / p10 / p90 over
    `replays` steps.  One JSON line per workload."""
    import numpy as np
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = "cuda:0"
    h = D.Handle(0)
    lines = []
    for cid, name in ((3, "ragged_B8192_T10-50_K10_tol1e-5"), (4, "dense_B16384_T50_K5_ckpt10")):
        print("bench: building workload %s" % name, file=sys.stderr, flush=True)
        d = W.make(cid)
        t = _tensors(d, dev)
        B = d["B"]
        row = dict(workload=name, B=B, T_max=d["T_max"], K=d["K"], tol=d["tol"], ckpt=d["ckpt"],
                   cost="dense" if d["cost_kind"] else "diag")
        for form, flags in (("persistent", D.NEED_GRAD | D.LPT | D.TUNED), ("plain", D.NEED_GRAD | D.PLAIN),
                            ("fp64", D.NEED_GRAD | D.LPT | D.TUNED | D.F64)):
            S = _solver(h, d, t, flags, dev)
            if form != "plain":
                row["launch_choice" if form == "persistent" else "launch_choice_fp64"] = S["tune"]()
            S["step"]()
            torch.cuda.synchronize()
            D.capture_begin(h, S["s"])
            S["step"]()
            g = D.capture_end(h, S["s"])
            graph = lambda: D.graph_launch(h, g, S["s"])  # noqa: E731
            graph()
            ev_g = pct(event_times(graph, S["s"], replays))
            S["step"]()
            ev_e = pct(event_times(S["step"], S["s"], replays))
            ev_f = pct(event_times(S["fwd"], S["s"], max(5, replays // 2)))
            st = S["out"]["st"].cpu().numpy().astype(np.uint32)
            its = (st >> 8) & 255
            row[form] = dict(graph_step_ms=ev_g, eager_step_ms=ev_e, fwd_ms=ev_f,
                             solves_per_s=B / (ev_g["median"] * 1e-3))
            if form == "persistent":
                Tb = d["T"].astype(np.float64)
                i = 1 if d["cost_kind"] else 0
                fl = Tb * (FLOP["init"][i] + its * FLOP["iter_stage"][i] + FLOP["tail"][i])
                ach = fl.sum() / (ev_f["median"] * 1e-3)
                row["roofline_fwd"] = dict(achieved=ach / 1e12, peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                                           frac=ach / PEAK_FP32, frac_vs_fp64_78_6=ach / PEAK_FP64,
                                           flop_fwd_total=float(fl.sum()),
                                           basis="per instance T_b (593 + k_b 27416 + 23478) diag / (593 + k_b "
                                                 "30204 + 23478) dense, k_b the iterations it used")
                row["iterations"] = dict(mean=float(its.mean()), converged=float(np.mean((st & 1) != 0)))
            D.graph_destroy(h, g)
            del S
            torch.cuda.synchronize()
        row["speedup_vs_plain_graph"] = row["plain"]["graph_step_ms"]["median"] / row["persistent"]["graph_step_ms"]["median"]
        row["speedup_vs_plain_eager"] = row["plain"]["eager_step_ms"]["median"] / row["persistent"]["graph_step_ms"]["median"]
        print(json.dumps(row), flush=True)
        lines.append(row)
    return lines


def tune_survey():
    """Forward time of every launch choice the autotuner considers, each
    pinned with dmpc_set_tuned and timed with HIP events (best of three after
    a warm-up), then dmpc_autotune's own pick, on the metric workload (B=4096,
    T=20, MLP cost), the ragged one (B=8192, T in 10..50) and the large dense
    one (B=16384, T=50, checkpoints).  Prints a markdown table."""
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = "cuda:0"
    h = D.Handle(0)
    wl = ((2, "B=4096 T=20 diag (MLP cost)"), (3, "B=8192 T=10..50 ragged"), (4, "B=16384 T=50 dense, ckpt 10"),
          (5, "B=256 T=50 hover-to-target"))
    print("| workload | form | instances/wave | waves/SIMD | grid | order | forward ms |")
    print("|---|---|---|---|---|---|---|")
    picks = []
    for cid, name in wl:
        if cid == 5:
            d = W.make_hover_target(256, 50)
        else:
            d = W.make(cid)
        t = _tensors(d, dev)
        S = _solver(h, d, t, D.NEED_GRAD | D.LPT | D.TUNED, dev)
        cands = [D.LaunchChoice(1, 0, 1, 0, 0.0)]
        for occ in (1, 2):
            for grid in (0, 1):
                for lpt in (0, 1):
                    cands.append(D.LaunchChoice(0, lpt, occ, grid, 0.0))
        for ipw in (2, 1):
            for lpt in (0, 1):
                cands.append(D.LaunchChoice(0, lpt, 1, 1, 0.0, ipw))
        for c in cands:
            D.set_tuned(h, S["cfg"], True, c)
            S["fwd"]()
            ms = min(event_times(S["fwd"], S["s"], 3))
            if c.plain:
                print("| %s | per-launch | - | - | - | - | %.3f |" % (name, ms), flush=True)
            else:
                print("| %s | persistent | %d | %d | %s | %s | %.3f |"
                      % (name, c.inst_per_wave, c.waves_per_simd,
                         "one wave per unit" if c.grid_mode else "resident + queue",
                         "longest first" if c.lpt else "queue", ms), flush=True)
        ch = S["tune"]()
        picks.append((name, ch))
        del S
        torch.cuda.synchronize()
    print()
    print("Choices dmpc_autotune stored:")
    print()
    for name, ch in picks:
        if ch["plain"]:
            print("- %s: per-launch form, %.3f ms" % (name, ch["ms"]))
        else:
            print("- %s: persistent, %d instance(s)/wave, %d wave(s)/SIMD, %s, %s, %.3f ms"
                  % (name, ch["inst_per_wave"], ch["waves_per_simd"],
                     "one wave per unit" if ch["grid_mode"] else "resident + queue",
                     "longest horizon first" if ch["lpt"] else "queue order", ch["ms"]))
    print()
    print("Kernel source hash %s." % kernel_source_hash(), flush=True)


def oracle_table(budget=3.0):
    """The FP64 oracle's time per workload on this host: forward on one thread
    and on the host threads this process may use (at most 16), the
    Riccati-adjoint backward and the dense-KKT backward (the verification
    path), each on a bounded sample of the workload's instances (repeated for
    about `budget` seconds) and scaled linearly to the batch (instances are
    independent).  Test infrastructure only: nothing here runs on the GPU.
    Prints one JSON line."""
    import numpy as np

    import oracle as orc
    import workloads as W
    P = orc.params_from(W.quad_params_f32())
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    nt = max(1, min(16, avail))
    rows = []
    for cid, n1, nall in ((0, 8, 8), (1, 64, 1024), (2, 64, 1024), (3, 64, 1024), (4, 32, 256)):
        d = W.make(cid) if cid != 4 else W.make(4, B=nall)
        B = W.CONFIGS[cid]["B"]

        def sub(n):
            return {k: d[k][:n] for k in ("x0", "Q", "p", "lo", "hi", "T", "grad_u")}

        def timed(fn):
            t0, reps = time.perf_counter(), 0
            while True:
                fn()
                reps += 1
                w = time.perf_counter() - t0
                if w >= budget or reps >= 200:
                    return w / reps

        a1, aa = sub(n1), sub(min(nall, d["B"]))
        fw = lambda a, t: orc.forward(P, a["x0"], a["Q"], a["p"], a["lo"], a["hi"], a["T"], K=d["K"], tol=d["tol"],
                                      nthreads=t)  # noqa: E731
        t1 = timed(lambda: fw(a1, 1)) / len(a1["T"])
        ta = timed(lambda: fw(aa, nt)) / len(aa["T"])
        f = fw(aa, nt)
        bw = lambda m: orc.backward(P, aa["x0"], aa["Q"], aa["p"], aa["lo"], aa["hi"], f["u"], f["x"], aa["grad_u"],
                                    T=aa["T"], method=m, nthreads=nt)  # noqa: E731
        tr = timed(lambda: bw(0)) / len(aa["T"])
        tk = timed(lambda: bw(1)) / len(aa["T"])
        rows.append(dict(cfg=cid, B=B, T_max=d["T_max"], K=d["K"],
                         fwd_1thread_s=t1 * B, fwd_all_s=ta * B, riccati_bwd_all_s=tr * B, dense_kkt_bwd_all_s=tk * B,
                         fwd_bwd_solves_per_s_all=1.0 / (ta + tr),
                         sample="forward on 1 thread: %d instances; the rest on %d threads: %d instances; per-instance "
                                "times scaled to B=%d" % (n1, nt, len(aa["T"]), B)))
        print("oracle cfg %d: fwd 1 thread %.3f s, fwd %d threads %.3f s, Riccati bwd %.3f s, dense-KKT bwd %.3f s "
              "(scaled to B=%d)" % (cid, t1 * B, nt, ta * B, tr * B, tk * B, B), file=sys.stderr, flush=True)
    print(json.dumps({"oracle_table": rows, "threads": nt, "host_cpu": cpu_model(), "host_nproc": os.cpu_count()}),
          flush=True)


def peaks(reps=20):
    """Measured ceilings on this GPU: the FP32 (single, unpacked: packed FP32
    is not built here) and FP64 FMA rates, every lane running eight
    independent FMA chains, with the chip full (16 waves per SIMD) and with
    one wave per SIMD (the forward kernel's occupancy at B = 4096); and the
    rate of a float4 device copy of 1 GiB (bytes read + written).  Median of
    `reps` launches, HIP events.  Prints one JSON line."""
    import ctypes as C

    import numpy as np
    import torch

    from paper_2605_29155_amd import build as _b
    L = C.CDLL(_b.PEAKS_LIB)
    L.peak_fma32.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.peak_fma64.argtypes = [C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_void_p]
    L.peak_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
    dev = "cuda:0"
    s = torch.cuda.Stream()
    sp = C.c_void_p(s.cuda_stream)
    out = {}
    iters = 2048
    cu = torch.cuda.get_device_properties(0).multi_processor_count
    for occ, blocks, threads in (("full", cu * 16, 256), ("1wave_per_simd", cu * 4, 64),
                                 ("2waves_per_simd", cu * 8, 64)):
        for name, fn, dt in (("fma_f32", L.peak_fma32, torch.float32), ("fma_f64", L.peak_fma64, torch.float64)):
            buf = torch.empty(blocks * threads, dtype=dt, device=dev)
            run = lambda: fn(blocks, threads, iters, C.c_void_p(buf.data_ptr()), sp)  # noqa: E731
            assert run() == 0
            ms = float(np.median(event_times(run, s, reps)))
            flop = 2.0 * 8 * 8 * iters * blocks * threads
            out["%s_%s" % (name, occ)] = dict(tflops=flop / (ms * 1e-3) / 1e12, ms=ms, flop=flop, blocks=blocks,
                                              threads=threads)
    n4 = (1 << 30) // 16
    src = torch.ones(n4 * 4, device=dev)
    dst = torch.empty_like(src)
    run = lambda: L.peak_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n4, cu * 64, sp)  # noqa: E731
    run()
    ms = float(np.median(event_times(run, s, reps)))
    out["copy"] = dict(gbps=2.0 * 16 * n4 / (ms * 1e-3) / 1e9, ms=ms, bytes=2 * 16 * n4)
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    out["published"] = dict(fp32_tflops=157.3, fp64_tflops=78.6, hbm_gbps=8000.0)
    print(json.dumps({"peaks": out, "compute_units": cu}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--latency", action="store_true",
                    help="forward / backward latency at the paper's Table I shapes (B 1 and 256, T 2, 10, 50) "
                         "on a hover-to-target workload; prints one JSON line with the table")
    ap.add_argument("--closed-loop", action="store_true",
                    help="receding-horizon control-step latency at B=1 (T 10, 20, 50; fixed K=5 and K<=30 with "
                         "tol 1e-5; cold, warm, warm+graph); prints one JSON line with the table")
    ap.add_argument("--shard", type=int, default=0, metavar="G",
                    help="one GPU's share of the metric workload split over G GPUs (B = 4096 / G, T = 20): "
                         "fwd+bwd step time of the tuned persistent form and of the per-launch form; prints one "
                         "JSON line")
    ap.add_argument("--configs", action="store_true",
                    help="fwd+bwd step of the ragged (B=8192) and large dense (B=16384, T=50) workloads, tuned "
                         "persistent and per-launch forms, eager and graph-captured; one JSON line each")
    ap.add_argument("--tune-survey", action="store_true",
                    help="forward time of every launch choice on the metric, ragged and dense workloads, and the "
                         "autotuner's pick; prints a markdown table")
    ap.add_argument("--peaks", action="store_true",
                    help="measured unpacked-FP32 and FP64 FMA rates and device-copy bandwidth; one JSON line")
    ap.add_argument("--oracle-table", action="store_true",
                    help="the FP64 oracle's forward (1 thread and all threads), Riccati-adjoint and dense-KKT "
                         "backward times per workload on this host (CPU only); prints one JSON line")
    ap.add_argument("--profile-short", action="store_true",
                    help="for counter collection: two direct fwd+bwd calls of the persistent form, then a "
                         "256 MiB device copy whose FETCH_SIZE / WRITE_SIZE calibrate the HBM counters")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the instances are independent and the layer has no "
              "cross-GPU step; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
    if a.oracle_table:
        oracle_table()
        return
    import torch
    dev = "cuda:0"
    if a.latency:
        print(json.dumps({"latency_table": latency_table(), "workload": "hover_to_random_target, K=5",
                          "paper_hardware": "NVIDIA RTX A6000 + Intel i9-13900K"}), flush=True)
        return
    if a.closed_loop:
        print(json.dumps({"closed_loop_latency": closed_loop_latency(), "workload": "hover_to_random_target, B=1"}),
              flush=True)
        return
    if a.configs:
        config_lines()
        return
    if a.peaks:
        peaks()
        return
    if a.tune_survey:
        tune_survey()
        return
    if a.shard > 0:
        Bs = 4096 // a.shard
        d, t = make_inputs(dev, Bs)
        res = run_gpu_bench(d, t, a.steps, a.warmup)
        per, pl = res["persistent"], res["plain"]
        print(json.dumps({"shard": dict(gpus=a.shard, B=Bs, T=d["T_max"], K=d["K"],
                                        ms_per_step=per["s_per_step"] * 1e3, solves_per_s=Bs / per["s_per_step"],
                                        fwd_ms=per["fwd_ms"], launch_choice=per["choice"],
                                        plain_ms_per_step=pl["s_per_step"] * 1e3)}),
              flush=True)
        return
    print("bench: building inputs (B=4096, T=20, MLP cost)", file=sys.stderr, flush=True)
    d, t = make_inputs(dev)
    if a.profile_short:
        profile_short(d, t)
        return
    print("bench: timing %d steps after %d warmup" % (a.steps, a.warmup), file=sys.stderr, flush=True)
    res = run_gpu_bench(d, t, a.steps, a.warmup)
    B, T, K = d["B"], d["T_max"], d["K"]
    f_fwd, f_bwd = flops_per_solve(T, K)
    per, pl = res["persistent"], res["plain"]
    value = B / per["s_per_step"]
    plain_value = B / pl["s_per_step"]
    achieved = f_fwd * B / (per["fwd_ms"] * 1e-3)
    kh = kernel_source_hash()
    ch = per["choice"]
    if ch["plain"]:
        form, kname = "per-launch (chosen by the autotuner), hipGraph fwd+bwd", "k_plain_riccati"
        traffic = None
    else:
        form = ("persistent (autotuner: %d wave(s)/SIMD, grid mode %d, %s order), hipGraph fwd+bwd"
                % (ch["waves_per_simd"], ch["grid_mode"], "longest-first" if ch["lpt"] else "queue"))
        ipw = ch.get("inst_per_wave", 4)
        kname = "k_fwd_persistent<false, %d, float, %d>" % (ch["waves_per_simd"], ipw)
        traffic = load_traffic(kh, B) if (ch["waves_per_simd"], ipw) == (1, 4) else None
    print("bench: torch steps through DMPCLayer", file=sys.stderr, flush=True)
    ts = torch_steps(d, t)
    import numpy as np
    line = {
        "metric": "fwd+bwd diff-MPC solves/s @B=4096,T=20 FP32 vs plain GPU; grad rel err",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": per["s_per_step"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64acc", "data": "synthetic",
        "config": {"workload": "diffmpc_quadrotor_B4096_T20_K5_mlpcost", "B": B, "T": T, "K": K,
                   "cost": "diag (MLP-emitted)", "form": form, "launch_choice": ch},
        "step_ms_events": {"persistent_graph": per["graph_step_ms"], "persistent_eager": per["eager_step_ms"],
                           "plain_graph": pl["graph_step_ms"], "plain_eager": pl["eager_step_ms"]},
        "fp64_form": {"graph_step_ms": res["fp64"]["graph_step_ms"], "fwd_ms": res["fp64"]["fwd_ms"],
                      "value": B / (res["fp64"]["graph_step_ms"]["median"] * 1e-3),
                      "launch_choice": res["fp64"]["choice"],
                      "note": "DMPC_F64: dynamics, linearisation, line search and stored trajectories in FP64"},
        "plain": {"value": plain_value, "ms_per_step": pl["s_per_step"] * 1e3, "form": "per-launch, eager",
                  "launches_fwd": pl["launches"], "speedup": value / plain_value,
                  "graph_value": B / (pl["graph_step_ms"]["median"] * 1e-3),
                  "speedup_vs_plain_graph": pl["graph_step_ms"]["median"] / per["graph_step_ms"]["median"]},
        "torch_step": {"layer_ms": ts["layer_ms"], "full_ms": ts["full_ms"],
                       "note": "DMPCLayer (autograd.Function) fwd + loss.backward, wall clock; full_ms includes "
                               "the cost MLP's forward and backward",
                       "layer_grad_equals_raw": bool(np.array_equal(ts["dp_layer"], per["dp"]))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32, "traffic": traffic,
                     "kernel": kname, "kernel_ms": per["fwd_ms"],
                     "kernel_ms_is": "median HIP-event time of the forward call (queue reset + forward kernel) on "
                                     "the stream it is launched on, 20 calls after the timed region",
                     "flop_per_solve_fwd": f_fwd, "frac_vs_fp64_78_6": achieved / PEAK_FP64},
        "kernel_source_hash": kh,
    }
    if not a.no_cpu:
        print("bench: CPU baseline leg (oracle)", file=sys.stderr, flush=True)
        cpu, acc = cpu_baseline_leg(d, res)
        line["cpu_baseline"] = cpu
        line["accuracy"] = acc
    else:
        line["cpu_baseline"] = None
    torch.cuda.synchronize()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
