#!/usr/bin/env python3
"""Throughput of the LKS forward + ALKS adjoint path on one MI355X.

One benchmark step is one design gradient of the steady 512x512 channel
(Re = 100, gamma a smoothed Gaussian field, 40000 LKS steps, the pressure-drop
objective, 40000 ALKS steps and the sensitivity), run on the FP32-deviation
path. The plain FP64 GPU path (same kernels instantiated in double) is timed
beside it, and the FP32 result is compared with it.

Prints one JSON line. MLUPS = nodes * (forward + adjoint steps) / time.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--fp64-steps", type=int, default=1)
    p.add_argument("--n-fwd", type=int, default=40000)
    p.add_argument("--n-adj", type=int, default=40000)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-steps", type=int, default=400)
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--batch-steps", type=int, default=2000)
    return p.parse_args()


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
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        J = None
        for _ in range(k):
            J = gradient(ctx, out)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k, J, out

    c32 = lks.LKS(wl, precision="fp32", device=dev)
    ty32 = c32.autotune(g, 200)
    ms32, J32, d32 = timed(c32, args.steps, args.warmup)
    c64 = lks.LKS(wl, precision="fp64", device=dev)
    ty64 = c64.autotune(g, 200)
    ms64, J64, d64 = timed(c64, args.fp64_steps, 0)

    upd = nodes * (wl.n_fwd + wl.n_adj)
    mlups32 = upd / (ms32 * 1e-3) / 1e6
    mlups64 = upd / (ms64 * 1e-3) / 1e6
    a, b = d32.cpu().numpy(), d64.cpu().numpy()
    err_grad = float(np.linalg.norm(a - b) / np.linalg.norm(b))
    err_J = abs(J32 - J64) / abs(J64)

    # dominant kernel: the ALKS step. Its average duration is measured on
    # this stream with events around a run of back-to-back adjoint steps
    # (the boundary pre-pass of each step included); algorithmic bytes per
    # node: read rho~, V (3 values) and u (2) and 1/(1+alpha), the node class
    # byte, write rho~, V (3) -> 9 * 4 + 1 = 37 B in FP32.
    nprobe = 4000
    out = torch.empty_like(g)
    c32.forward(g, wl.n_fwd)
    c32.backward(1.0, out, 10)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    c32.adjoint_advance(1.0, nprobe, None)
    e1.record()
    torch.cuda.synchronize()
    alks_us = e0.elapsed_time(e1) * 1e3 / nprobe
    bytes_per_node = 37
    achieved = bytes_per_node * nodes / (alks_us * 1e-6) / 1e9
    roofline = {"bound": "hbm", "kernel": "alks_step_kernel<float>", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None, "avg_launch_us": alks_us,
                "bytes_per_node": bytes_per_node, "nodes_per_launch": nodes}

    batched = None if args.no_batch else batched_bench(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(wl, args.cpu_sample_steps)

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
                               "field (sigma=8), pressure-drop objective",
                   "nx": wl.nx, "ny": wl.ny, "n_fwd": wl.n_fwd, "n_adj": wl.n_adj,
                   "precision": "fp32 state (rho-1), fp64 objective and sensitivity",
                   "tile_rows": {"fp32": ty32, "fp64": ty64}},
        "gradients_per_s": 1e3 / ms32,
        "fp64_gpu": {"value": mlups64, "unit": "MLUPS", "ms_per_step": ms64,
                     "gradients_per_s": 1e3 / ms64},
        "speedup_vs_fp64_gpu": ms64 / ms32,
        "fp32_vs_fp64_rel_error": {"J": err_J, "dJdgamma_l2": err_grad},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "batched_64_designs": batched,
    }
    print(json.dumps(line), flush=True)


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
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    b.run(gs, outs, 0, n)
    e1.record()
    torch.cuda.synchronize()
    adj_us = e0.elapsed_time(e1) * 1e3 / n
    achieved = 37 * nodes / (adj_us * 1e-6) / 1e9
    return {"designs": 64, "nodes": nodes, "n_fwd": n, "n_adj": n, "ms_per_batch": ms,
            "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
            "gradients_per_s": 64 * 1e3 / ms, "tile_rows": ty,
            "roofline": {"bound": "hbm", "kernel": "alks_step_batch_kernel<float>",
                         "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "avg_launch_us": adj_us,
                         "bytes_per_node": 37, "nodes_per_launch": nodes}}


def cpu_baseline(wl, n):
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: n forward and n adjoint steps of the 512x512 grid."""
    import numpy as np
    import oracle as O
    pb = O.Problem(wl)
    alpha, _, B, _ = O.coefficients(pb, wl.gamma)
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
    nodes = wl.nx * wl.ny
    mlups = nodes * 2 * n / (t2 - t0) / 1e6
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": mlups, "unit": "MLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{wl.nx}x{wl.ny}, {n} forward + {n} adjoint FP64 steps "
                      f"({t1 - t0:.1f} s + {t2 - t1:.1f} s)",
            "forward_mlups": nodes * n / (t1 - t0) / 1e6,
            "adjoint_mlups": nodes * n / (t2 - t1) / 1e6}


if __name__ == "__main__":
    main()
