#!/usr/bin/env python3
"""Throughput of the LKS forward + ALKS adjoint path on one MI355X.

One benchmark step is one design gradient of the steady 512x512 channel
(Re = 100, gamma a smoothed Gaussian field, 40000 LKS steps, the pressure-drop
objective, 40000 ALKS steps and the sensitivity), run on the FP32-deviation
path. The plain FP64 GPU path (the same kernels instantiated in double, one
step per launch) is timed beside it, and the FP32 result is compared with it.

Further sections of the same JSON line (not the headline value):
  batched_64_designs      64 independent steady designs of uneven size, one
                          launch per step for all of them, HIP graph replay;
  unsteady_thermal_1024x512  the checkpointed unsteady thermal sweep
                          (20000 steps, K from a memory budget);
  duct3d_256x128x128      the D3Q19 heated-block duct (5000 steps,
                          checkpointed).

Prints one JSON line. MLUPS = nodes * (forward + adjoint steps) / time; the
replayed forward steps of checkpointed sweeps are cost, not updates.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "alks_step_512x512_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_2411_03090_amd", "csrc", "lks_kernels.hip")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--fp64-steps", type=int, default=1)
    p.add_argument("--n-fwd", type=int, default=40000)
    p.add_argument("--n-adj", type=int, default=40000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-steps", type=int, default=2500)
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--batch-steps", type=int, default=2000)
    p.add_argument("--no-unsteady", action="store_true")
    p.add_argument("--unsteady-steps", type=int, default=20000)
    p.add_argument("--no-large", action="store_true")
    p.add_argument("--large-steps", type=int, default=2000)
    p.add_argument("--no-exchanger", action="store_true")
    p.add_argument("--no-sink", action="store_true")
    p.add_argument("--sink-steps", type=int, default=50000)
    p.add_argument("--exchanger-steps", type=int, default=20000)
    p.add_argument("--no-3d", action="store_true")
    p.add_argument("--steps-3d", type=int, default=5000)
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 256 MiB device copy (counter calibration)")
    return p.parse_args()


def ev():
    import torch
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def rel(a, b):
    import numpy as np
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the path is a single-GPU kernel sweep and no "
              "multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_03090_amd import lks, workloads as W

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
        return
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0,
                              n_fwd=args.n_fwd, n_adj=args.n_adj)
    nodes = wl.nx * wl.ny
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)

    def gradient(ctx, out):
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        ctx.backward(1.0, out, wl.n_adj)
        return J

    def timed(ctx, k, w):
        out = torch.empty_like(g)
        for _ in range(w):
            gradient(ctx, out)
        torch.cuda.synchronize()
        e0 = ev()
        J = None
        for _ in range(k):
            J = gradient(ctx, out)
        e1 = ev()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, J, out

    c32 = lks.LKS(wl, precision="fp32", device=dev)
    c32.autotune(g, 200)
    shape32 = c32.launch_shape()
    ms32, J32, d32 = timed(c32, args.steps, args.warmup)
    # the plain FP64 path: one step per launch, tile height tuned
    c64 = lks.LKS(wl, precision="fp64", device=dev)
    c64.autotune(g, 200)
    shape64 = c64.launch_shape()
    ms64, J64, d64 = timed(c64, args.fp64_steps, 0)

    upd = nodes * (wl.n_fwd + wl.n_adj)
    mlups32 = upd / (ms32 * 1e-3) / 1e6
    mlups64 = upd / (ms64 * 1e-3) / 1e6
    err_grad = rel(d32.cpu().numpy(), d64.cpu().numpy())
    err_J = abs(J32 - J64) / abs(J64)
    # final forward fields of the last gradient of each context
    err_fields = {n: rel(c32.read(n).cpu().numpy(), c64.read(n).cpu().numpy())
                  for n in ("drho", "ux", "uy")}

    roofline = alks_roofline(c32, g, wl, nodes, shape32)
    batched = None if args.no_batch else batched_bench(args, dev)
    unsteady = None if args.no_unsteady else unsteady_bench(args, dev)
    large = None if args.no_large else large_bench(args, dev)
    exchanger = None if args.no_exchanger else exchanger_bench(args, dev)
    sink = None if args.no_sink else sink_bench(args, dev)
    duct = None if args.no_3d else duct3d_bench(args, dev)
    cpu = None if args.no_cpu_baseline else cpu_baseline(wl, args.cpu_sample_steps)

    line = {
        "metric": "MLUPS forward+adjoint and design gradients/sec vs plain FP64 GPU at stated error",
        "value": mlups32,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "steady channel 512x512 D2Q9, Re=100, gamma smoothed Gaussian "
                               "field (sigma=8), pressure-drop objective, one gradient",
                   "nx": wl.nx, "ny": wl.ny, "n_fwd": wl.n_fwd, "n_adj": wl.n_adj,
                   "precision": "fp32 state (rho-1), fp64 objective and sensitivity",
                   "launch_shape": {p: {"tile_rows": s[0], "forward_steps_per_launch": s[1],
                                        "adjoint_steps_per_launch": s[2]}
                                    for p, s in (("fp32", shape32), ("fp64", shape64))}},
        "gradients_per_s": 1e3 / ms32,
        "fp64_gpu": {"value": mlups64, "unit": "MLUPS", "ms_per_step": ms64,
                     "gradients_per_s": 1e3 / ms64},
        "speedup_vs_fp64_gpu": ms64 / ms32,
        "fp32_vs_fp64_rel_error": {"J": err_J, "dJdgamma_l2": err_grad, "fields_l2": err_fields},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_64_designs": batched,
        "unsteady_thermal_1024x512": unsteady,
        "steady_2048x2048": large,
        "heat_exchanger_201x201": exchanger,
        "heat_sink_141x161": sink,
        "duct3d_256x128x128": duct,
    }
    print(json.dumps(line), flush=True)


def alks_roofline(ctx, g, wl, nodes, shape):
    """Dominant kernel: the ALKS step. Its average launch duration is
    measured with events on the context's stream around a run of
    back-to-back adjoint steps. Algorithmic bytes per node update: read
    rho~, V (3 values), u (2) and 1/(1+alpha) and the node-class byte, write
    rho~, V (3): 9 * 4 + 1 = 37 B in FP32."""
    import torch
    nprobe = 4000
    out = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    ctx.backward(1.0, out, 10)
    torch.cuda.synchronize()
    e0 = ev()
    ctx.adjoint_advance(1.0, nprobe, None)
    e1 = ev()
    torch.cuda.synchronize()
    ty, spl = shape[0], shape[2]
    step_us = e0.elapsed_time(e1) * 1e3 / nprobe
    launch_us = step_us * spl
    bytes_per_node = 37
    algo = bytes_per_node * nodes * spl                  # bytes per launch
    achieved = algo / (launch_us * 1e-6) / 1e9
    kernel = (f"alks_step2_kernel<float, false, {ty}>" if spl == 2
              else f"alks_step_kernel<float, false, {ty}>")
    return {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic_per_launch(kernel), "avg_launch_us": launch_us,
            "bytes_per_node_update": bytes_per_node, "node_updates_per_launch": nodes * spl,
            "algorithmic_bytes_per_launch": algo}


def traffic_per_launch(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, each scaled by the reading for a plain
    copy of known size), or None when it was taken on other kernel source or
    another kernel."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    sha = hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()
    k = t.get("kernels", {}).get(kernel)
    if t.get("source_sha256") != sha or k is None:
        return None
    return k["fetch_kib"] * 1024 / t["fetch_factor"] + k["write_kib"] * 1024 / t["write_factor"]


def batched_bench(args, dev):
    """64 independent steady designs, edge lengths from {128,...,512} and
    Re in [10, 200], forward + adjoint of all designs with one launch per
    step, replayed as a HIP graph (FP32 state, FP64 J and dJ/dgamma)."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.batch_steps
    wls = W.batch_designs(64, n_steps=n)
    nodes = sum(w.nx * w.ny for w in wls)
    b = lks.Batch(wls, precision="fp32", device=dev)
    gs = [torch.tensor(w.gamma.reshape(-1), dtype=torch.float64, device=dev) for w in wls]
    outs = [torch.empty_like(x) for x in gs]
    ty = b.autotune(gs, outs, 50)
    b.run(gs, outs, n, n)                                   # warm-up, builds the graph
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run(gs, outs, n, n)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    # batched ALKS step alone: a run with no forward steps and n adjoint steps
    b.run(gs, outs, 0, n)
    torch.cuda.synchronize()
    e0 = ev()
    b.run(gs, outs, 0, n)
    e1 = ev()
    torch.cuda.synchronize()
    adj_us = e0.elapsed_time(e1) * 1e3 / n
    achieved = 37 * nodes / (adj_us * 1e-6) / 1e9
    return {"designs": 64, "nodes": nodes, "n_fwd": n, "n_adj": n, "ms_per_batch": ms,
            "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
            "gradients_per_s": 64 * 1e3 / ms, "tile_rows": ty,
            "roofline": {"bound": "hbm", "kernel": f"alks_step_batch_kernel<float, false, {ty}>",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "avg_launch_us": adj_us,
                         "bytes_per_node_update": 37, "node_updates_per_launch": nodes}}


def _checkpointed(ctx_fp32, ctx_fp64, g, nodes, n):
    """Time one gradient on each context; the checkpointed sweep replays
    the forward segments inside the backward call."""
    import numpy as np
    import torch
    res = {}
    outs = {}
    for name, c in (("fp32", ctx_fp32), ("fp64", ctx_fp64)):
        out = torch.empty_like(g)
        torch.cuda.synchronize()
        e0 = ev()
        c.forward(g)
        J = c.objective()
        e1 = ev()
        c.backward(1.0, out)
        e2 = ev()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e2)
        rep = c.memory_report()
        res[name] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                     "gradients_per_s": 1e3 / ms, "forward_ms": e0.elapsed_time(e1),
                     "backward_ms": e1.elapsed_time(e2), "K": rep["K"],
                     "checkpoint_GiB": rep["ckpt_bytes"] / 2 ** 30, "J": J}
        outs[name] = out.cpu().numpy()
    res["speedup_fp32_vs_fp64"] = res["fp64"]["ms_per_gradient"] / res["fp32"]["ms_per_gradient"]
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {
        "J": abs(res["fp32"]["J"] - J64) / abs(J64) if J64 else None,
        "dJdgamma_l2": rel(outs["fp32"], outs["fp64"]) if np.any(outs["fp64"]) else None}
    return res, outs["fp32"]


def unsteady_bench(args, dev):
    """1024x512 unsteady forced convection (Re = 200, Pr = 6, oscillating
    inflow), time-averaged heat objective, 20000 steps; the adjoint replays
    the forward from checkpoints every K levels, K the largest that fits the
    memory budget (4 GiB FP32, 8 GiB FP64)."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.unsteady_steps
    wl = W.unsteady_thermal_channel(1024, 512, n_steps=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    c32 = lks.LKS(wl, precision="fp32", mem_budget=4 * 2 ** 30, device=dev)
    c64 = lks.LKS(wl, precision="fp64", mem_budget=8 * 2 ** 30, device=dev)
    for c in (c32, c64):
        c.autotune(g, 100)
    res, _ = _checkpointed(c32, c64, g, wl.nx * wl.ny, n)
    res["tile_rows"] = {"fp32": c32.launch_shape()[0], "fp64": c64.launch_shape()[0]}
    res.update({"nodes": wl.nx * wl.ny, "steps": n, "budget_GiB": {"fp32": 4, "fp64": 8}})
    del c32, c64
    torch.cuda.empty_cache()
    return res


def large_bench(args, dev):
    """The headline's steady channel at 2048x2048 (Re = 100, the same gamma
    recipe), n + n steps in FP32, autotuned: enough tiles to fill the chip,
    so the ALKS kernel is measured against HBM bandwidth rather than launch
    latency."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.large_steps
    wl = W.steady_channel_grf(2048, 2048, Re=100.0, sigma=8.0, seed=0, n_fwd=n, n_adj=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    nodes = wl.nx * wl.ny
    c = lks.LKS(wl, precision="fp32", device=dev)
    c.autotune(g, 50)
    shape = c.launch_shape()
    out = torch.empty_like(g)
    torch.cuda.synchronize()
    e0 = ev()
    c.forward(g, n)
    c.objective()
    c.backward(1.0, out, n)
    e1 = ev()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    res = {"mlups": nodes * 2 * n / (ms * 1e-3) / 1e6, "ms_per_gradient": ms,
           "n_fwd": n, "n_adj": n, "nodes": nodes,
           "launch_shape": {"tile_rows": shape[0], "forward_steps_per_launch": shape[1],
                            "adjoint_steps_per_launch": shape[2]},
           "roofline": alks_roofline(c, g, wl, nodes, shape)}
    res["roofline"]["traffic"] = None   # counters are taken on the 512x512 grid
    del c
    torch.cuda.empty_cache()
    return res


def exchanger_bench(args, dev):
    """Steady heat exchanger 201x201 (Re = 100, Pr = 6, heat source with
    beta_max = 0.1 in the solid, heat-exchange objective), n + n steps, one
    gradient in FP32 and in FP64."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.exchanger_steps
    wl = W.heat_exchanger(n=201, n_fwd=n, n_adj=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    nodes = wl.nx * wl.ny
    res, outs = {}, {}
    for prec in ("fp32", "fp64"):
        c = lks.LKS(wl, precision=prec, device=dev)
        c.autotune(g, 100)
        out = torch.empty_like(g)
        c.forward(g, 200)                                   # warm-up
        torch.cuda.synchronize()
        e0 = ev()
        c.forward(g, n)
        J = c.objective()
        c.backward(1.0, out, n)
        e1 = ev()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        res[prec] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                     "gradients_per_s": 1e3 / ms, "J": J}
        outs[prec] = out.cpu().numpy()
        del c
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {"J": abs(res["fp32"]["J"] - J64) / abs(J64),
                                     "dJdgamma_l2": rel(outs["fp32"], outs["fp64"])}
    res.update({"nodes": nodes, "n_fwd": n, "n_adj": n, "beta_max": wl.beta_max})
    torch.cuda.empty_cache()
    return res


def sink_bench(args, dev):
    """Transient natural-convection heat sink 141x161 (Ra = 2e5, Pr = 6,
    K_s = 10 K_f, heat flux 0.01 on the heated boundary), mean heated
    temperature averaged over n steps, whole trajectory kept; the adjoint in
    the exact mode, whose transposed conductivity term stays bounded at this
    contrast (the paper's form is reported beside it)."""
    import numpy as np
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.sink_steps
    wl = W.heat_sink(n_steps=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    nodes = wl.nx * wl.ny
    res, outs = {}, {}
    for prec, mode in (("fp32", "exact"), ("fp64", "exact"), ("fp32", "paper")):
        wl.adjoint_mode = mode
        c = lks.LKS(wl, precision=prec, device=dev)
        c.autotune(g, 100)
        out = torch.empty_like(g)
        torch.cuda.synchronize()
        e0 = ev()
        c.forward(g)
        J = c.objective()
        c.backward(1.0, out)
        e1 = ev()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        o = out.cpu().numpy()
        key = prec if mode == "exact" else "fp32_paper_mode"
        res[key] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                    "gradients_per_s": 1e3 / ms, "J": J,
                    "dJdgamma_finite": bool(np.isfinite(o).all()),
                    "dJdgamma_max_abs": float(np.abs(o).max()) if np.isfinite(o).all() else None}
        outs[key] = o
        del c
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {"J": abs(res["fp32"]["J"] - J64) / abs(J64),
                                     "dJdgamma_l2": rel(outs["fp32"], outs["fp64"])}
    res.update({"nodes": nodes, "steps": n, "adjoint_mode": "exact"})
    torch.cuda.empty_cache()
    return res


def duct3d_bench(args, dev):
    """D3Q19 256x128x128 duct with a heated block (Re = 100, Pr = 0.71),
    time-averaged heat objective, 5000 steps, checkpointed (16 GiB FP32,
    32 GiB FP64 budgets; the whole trajectory would take 335 GB in FP32)."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.steps_3d
    wl = W.heated_block_duct(n_steps=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    c32 = lks.LKS(wl, precision="fp32", mem_budget=16 * 2 ** 30, device=dev)
    c64 = lks.LKS(wl, precision="fp64", mem_budget=32 * 2 ** 30, device=dev)
    nodes = wl.nx * wl.ny * wl.nz
    res, grad16 = _checkpointed(c32, c64, g, nodes, n)
    res.update({"nodes": nodes, "steps": n, "budget_GiB": {"fp32": 16, "fp64": 32}})
    del c32, c64
    torch.cuda.empty_cache()
    # the same gradient in 4 GiB: two-level checkpoints do not fit, binomial
    # snapshots recompute more forward steps
    cb = lks.LKS(wl, precision="fp32", mem_budget=4 * 2 ** 30, device=dev)
    out = torch.empty_like(g)
    torch.cuda.synchronize()
    e0 = ev()
    cb.forward(g)
    cb.objective()
    e1 = ev()
    cb.backward(1.0, out)
    e2 = ev()
    torch.cuda.synchronize()
    info = cb.checkpoint_info()
    ms = e0.elapsed_time(e2)
    res["fp32_4GiB"] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                        "forward_ms": e0.elapsed_time(e1), "backward_ms": e1.elapsed_time(e2),
                        "scheme": info["scheme"], "snapshots": info["count"],
                        "replay_steps": info["replay_steps"],
                        "workspace_GiB": cb.workspace_size() / 2 ** 30,
                        "dJdgamma_bitwise_equal_to_16GiB_run":
                            bool((out.cpu().numpy() == grad16).all())}
    del cb
    torch.cuda.empty_cache()
    return res


def copy_calibration(dev):
    """A plain 256 MiB device-to-device copy: under rocprofv3 --pmc its
    FETCH_SIZE and WRITE_SIZE give the scale of the counters."""
    import torch
    n = 64 * 2 ** 20
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": 4 * n, "copies": 3}), flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_sample(O, pb, alpha, B, n):
    """n forward and n adjoint oracle steps of the workload; (forward s,
    adjoint s)."""
    s = O.init_state(pb, 1.0)
    for _ in range(5):
        s = O.lks_step(pb, alpha, B, 1.0, s)
    t0 = time.perf_counter()
    for _ in range(n):
        s = O.lks_step(pb, alpha, B, 1.0, s)
    t1 = time.perf_counter()
    adj = pb.zeros(O.N_ADJ_FIELDS)
    for _ in range(n):
        adj = O.alks_step(pb, alpha, B, s, s, adj, 1.0, 0.0)
    t2 = time.perf_counter()
    return t1 - t0, t2 - t1


def cpu_baseline(wl, n, n_one=None):
    """The FP64 oracle (gcc -O3, OpenMP) on the host cores, on a bounded
    sample of the same workload: n forward and n adjoint steps of the grid on
    every thread OpenMP uses, and a smaller sample on one thread."""
    import oracle as O
    pb = O.Problem(wl)
    alpha, _, B, _ = O.coefficients(pb, wl.gamma)
    nodes = wl.nx * wl.ny
    threads = O.max_threads()
    tf, ta = _oracle_sample(O, pb, alpha, B, n)
    mlups = nodes * 2 * n / (tf + ta) / 1e6
    n1 = n_one if n_one is not None else max(20, n // 10)
    O.set_threads(1)
    try:
        tf1, ta1 = _oracle_sample(O, pb, alpha, B, n1)
    finally:
        O.set_threads(threads)
    return {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{wl.nx}x{wl.ny}, {n} forward + {n} adjoint FP64 steps on {threads} "
                      f"threads ({tf:.1f} s + {ta:.1f} s)",
            "cpu_model": _cpu_model(), "nproc": os.cpu_count(), "build": "gcc -O3 -fopenmp",
            "forward_mlups": nodes * n / tf / 1e6, "adjoint_mlups": nodes * n / ta / 1e6,
            "gradients_per_s_extrapolated": mlups * 1e6 / (nodes * (wl.n_fwd + wl.n_adj)),
            "one_thread": {"value": nodes * 2 * n1 / (tf1 + ta1) / 1e6, "unit": "MLUPS",
                           "sample": f"{n1} forward + {n1} adjoint steps on 1 thread "
                                     f"({tf1:.1f} s + {ta1:.1f} s)"}}


if __name__ == "__main__":
    main()
