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
PEAK_ALU = 78.6e12   # 256 CU x 4 SIMD x 16 lanes x 2 FLOP x 2.4 GHz, unpacked FP32 FMA = FP64 FMA rate
PEAK_FP32_PACKED = 157.3e12
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


def run_gpu_bench(d, t, steps, warmup):
    import torch

    import paper_2605_29155_amd as D
    import workloads as W
    dev = t["x0"].device
    B, Tm, K = d["B"], d["T_max"], d["K"]
    h = D.Handle(0)
    params = D.quad_params(W.quad_params_f32())
    out = {}
    for form in ("persistent", "plain"):
        # the headline form uses the launch the autotuner picks for this shape
        flags = D.NEED_GRAD | (D.PLAIN if form == "plain" else D.LPT | D.TUNED)
        cfg = D.make_config(B, Tm, D.COST_DIAG, K, 0.0, flags)
        ws = D.alloc_workspace(cfg, dev)
        u = torch.empty(B, Tm, 4, device=dev)
        x = torch.empty(B, Tm, 13, device=dev)
        st = torch.empty(B, dtype=torch.int32, device=dev)
        gQ, gp, gx0 = torch.empty_like(t["Q"]), torch.empty_like(t["p"]), torch.empty_like(t["x0"])
        s = torch.cuda.Stream()

        def step():
            D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws, None, s)
            D.backward_raw(h, cfg, params, None, None, None, None, ws, t["grad_u"], None, gQ, gp, gx0, s)

        choice = None
        if form == "persistent":
            with torch.cuda.stream(s):
                choice = D.autotune(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws,
                                    s).as_dict()
        with torch.cuda.stream(s):
            step()
        torch.cuda.synchronize()
        launches = None
        if form == "persistent":
            # graph of the whole fwd+bwd step
            D.capture_begin(h, s)
            step()
            g = D.capture_end(h, s)
            run = lambda: D.graph_launch(h, g, s)  # noqa: E731
        else:
            D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws, None, s)
            launches = h.launch_count() + 1
            run = step
        for _ in range(warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        # dominant kernel: the forward, timed by HIP events on its own stream
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fwd_ms = []
        for _ in range(max(3, min(steps, 10))):
            e0.record(s)
            D.forward_raw(h, cfg, params, t["x0"], t["Q"], t["p"], t["lo"], t["hi"], None, u, x, st, ws, None, s)
            e1.record(s)
            D.backward_raw(h, cfg, params, None, None, None, None, ws, t["grad_u"], None, gQ, gp, gx0, s)
            e1.synchronize()
            fwd_ms.append(e0.elapsed_time(e1))
        torch.cuda.synchronize()
        out[form] = dict(s_per_step=dt, fwd_ms=sorted(fwd_ms)[len(fwd_ms) // 2], launches=launches, choice=choice,
                         u=u.cpu().numpy(), x=x.cpu().numpy(), status=st.cpu().numpy().astype("uint32"),
                         dQ=gQ.cpu().numpy(), dp=gp.cpu().numpy(), dx0=gx0.cpu().numpy())
        if form == "persistent":
            D.graph_destroy(h, g)
    return out


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


def cpu_baseline_leg(d, gpu, nsample=64):
    """Oracle on the host: time fwd + Riccati-adjoint bwd of the full batch on
    all host cores, and check the kernel on a sample with its decisions
    replayed (needs the decision log: one extra kernel run)."""
    import numpy as np
    import torch

    import oracle as orc
    import paper_2605_29155_amd as D
    import workloads as W
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import oracle_replay, rel, run_gpu
    P = orc.params_from(W.quad_params_f32())
    nthreads = min(16, os.cpu_count() or 1)
    # repeat the full batch until about 10 s of wall time have been spent
    t0 = time.perf_counter()
    reps = 0
    while True:
        f = orc.forward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], d["T"], K=d["K"], nthreads=nthreads)
        orc.backward(P, d["x0"], d["Q"], d["p"], d["lo"], d["hi"], f["u"], f["x"], d["grad_u"], T=d["T"],
                     nthreads=nthreads)
        reps += 1
        wall = time.perf_counter() - t0
        if wall >= 10.0 or reps >= 60:
            break
    cpu = dict(value=reps * d["B"] / wall, unit="solves/s", cores=nthreads, kind="oracle",
               sample="full batch B=%d T=%d K=%d repeated %d times, FP64 forward + Riccati-adjoint backward, "
                      "%.1f s wall" % (d["B"], d["T_max"], d["K"], reps, wall))
    # accuracy on a sample, decisions replayed
    idx = np.arange(0, d["B"], d["B"] // nsample)[:nsample]
    g = run_gpu(d, lpt=True)
    o = oracle_replay(d, g, idx=idx)
    sel = lambda a: a[idx]  # noqa: E731
    acc = dict(sample=len(idx),
               u_rel_max=float(rel(sel(g["u"]), o["replay"]["u"]).max()),
               dQ_rel_max=float(rel(sel(g["dQ"]), o["bwd"]["dQ"]).max()),
               dp_rel_max=float(rel(sel(g["dp"]), o["bwd"]["dp"]).max()),
               dx0_rel_max=float(rel(sel(g["dx0"]), o["bwd"]["dx0"]).max()))
    # the timed persistent run and the decision-logged run must agree exactly
    acc["bench_run_matches_logged_run"] = bool(np.array_equal(gpu["persistent"]["u"], g["u"]))
    torch.cuda.synchronize()
    del D
    return cpu, acc


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
    ap.add_argument("--profile-short", action="store_true",
                    help="for counter collection: two direct fwd+bwd calls of the persistent form, then a "
                         "256 MiB device copy whose FETCH_SIZE / WRITE_SIZE calibrate the HBM counters")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the instances are independent and the layer has no "
              "cross-GPU step; --gpus %d is not supported" % a.gpus, file=sys.stderr)
        sys.exit(2)
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
    per = res["persistent"]
    value = B / per["s_per_step"]
    plain_value = B / res["plain"]["s_per_step"]
    achieved = f_fwd * B / (per["fwd_ms"] * 1e-3)
    kh = kernel_source_hash()
    ch = per["choice"]
    if ch["plain"]:
        form, kname = "per-launch (chosen by the autotuner), hipGraph fwd+bwd", "k_plain_riccati"
        traffic = None
    else:
        form = ("persistent (autotuner: %d wave(s)/SIMD, grid mode %d, %s order), hipGraph fwd+bwd"
                % (ch["waves_per_simd"], ch["grid_mode"], "longest-first" if ch["lpt"] else "queue"))
        kname = "k_fwd_persistent<false, %d>" % ch["waves_per_simd"]
        traffic = load_traffic(kh, B) if ch["waves_per_simd"] == 1 else None
    line = {
        "metric": "fwd+bwd diff-MPC solves/s @B=4096,T=20 FP32 vs plain GPU; grad rel err",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": per["s_per_step"] * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64acc", "data": "synthetic",
        "config": {"workload": "diffmpc_quadrotor_B4096_T20_K5_mlpcost", "B": B, "T": T, "K": K,
                   "cost": "diag (MLP-emitted)", "form": form, "launch_choice": ch},
        "plain": {"value": plain_value, "ms_per_step": res["plain"]["s_per_step"] * 1e3,
                  "launches_fwd": res["plain"]["launches"], "speedup": value / plain_value},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_ALU / 1e12, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU, "traffic": traffic,
                     "kernel": kname, "kernel_ms": per["fwd_ms"],
                     "flop_per_solve_fwd": f_fwd, "frac_vs_fp32_packed": achieved / PEAK_FP32_PACKED},
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
