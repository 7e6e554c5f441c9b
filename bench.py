#!/usr/bin/env python3
"""Throughput of the LKS forward + ALKS adjoint path on one MI355X.

One benchmark step is one design gradient of the steady 512x512 channel
(Re = 100, gamma a smoothed Gaussian field, 40000 LKS steps, the pressure-drop
objective, 40000 ALKS steps and the sensitivity). Three paths compute it:
  fp64   the plain FP64 GPU path (the same kernels instantiated in double);
  fp32   the FP32-deviation path (state in float, density as rho - 1,
         objective and sensitivity in double);
  mixed  the forward sweep in FP64 and the adjoint sweep in FP32.
The headline value is the fastest path whose error against the plain FP64
path stays within the stated bounds (fields 1e-5, J and dJ/dgamma 1e-3,
relative L2); the others are reported beside it.

Further sections of the same JSON line (not the headline value):
  batched_64_designs        64 independent steady designs of uneven size, one
                            launch per step for all, HIP graph replay;
  steady_2048x2048          the headline's recipe at 16x the nodes;
  unsteady_thermal_1024x512 the checkpointed unsteady thermal sweep;
  heat_exchanger_201x201    the steady heat exchanger (heat source);
  heat_sink_141x161         the transient natural-convection heat sink;
  duct3d_256x128x128        the D3Q19 heated-block duct, checkpointed.

Rooflines. Every step is a memory-bound gather, so each section reports the
HBM roofline of its dominant kernel: algorithmic bytes per launch (bytes per
lattice update x updates per launch) over the average launch duration measured
with HIP events on the context's stream. The algorithmic bytes per update
read the state once and write it once, with gamma the only static field and
an FP64 sensitivity accumulator read and written once per update where the
sweep accumulates it (ALGO_BYTES). The library's own accounting (the adjoint
state kept as equilibrium coefficients, 1/(1 + alpha) and the node-class byte
read in place of gamma) is reported beside it (LIB_BYTES), and so are the HBM
bytes the rocprofv3 counters FETCH_SIZE and WRITE_SIZE measured for the same
kernel and launch shape (profiles/hbm_traffic.json), when they were taken on
the current kernel sources.

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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.json")
CSRC = os.path.join(ROOT, "paper_2411_03090_amd", "csrc")
KERNEL_SOURCES = ("lks_kernels.hip", "lks_kernels3d.hip", "lks_device.h")
SECTIONS = ("headline", "batch", "ubatch", "large", "unsteady", "exchanger", "sink", "duct3d")
BOUND_FIELDS, BOUND_GRAD = 1e-5, 1e-3

# algorithmic bytes per lattice update, (lattice/physics, sweep) -> (FP32, FP64):
# forward: the state read and written (2D 7 values, thermal 9, 3D thermal 11);
# steady adjoint: 6 adjoint moments in and out, u (2) and gamma; unsteady
# thermal adjoint: 9 (3D 14) moments in and out, u and T and gamma, plus the
# FP64 sensitivity accumulator read and written
ALGO_BYTES = {("2d", "fwd"): (28, 56), ("2d", "adj_steady"): (60, 120),
              ("2d_thermal", "fwd"): (36, 72), ("2d_thermal", "adj_unsteady"): (104, 192),
              ("3d_thermal", "fwd"): (44, 88), ("3d_thermal", "adj_unsteady"): (148, 280)}
# the library's bytes per update: the adjoint state as the equilibrium
# coefficients (rho~, V, Theta), 1/(1 + alpha), B, 3 alpha', B' and the
# node-class byte where the kernels read them
LIB_BYTES = {("2d", "fwd"): (29, 57), ("2d", "adj_steady"): (37, 73),
             ("2d_thermal", "fwd"): (41, 81), ("2d_thermal", "adj_unsteady"): (77, 137),
             ("3d_thermal", "fwd"): (49, 97), ("3d_thermal", "adj_unsteady"): (89, 161)}


def parse(argv=None):
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
    p.add_argument("--no-ubatch", action="store_true")
    p.add_argument("--ubatch-steps", type=int, default=2000)
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
    p.add_argument("--probe-steps", type=int, default=4000,
                   help="steps timed back to back for each roofline measurement")
    p.add_argument("--only", default="",
                   help="comma-separated sections to run (default: all): " + ",".join(SECTIONS))
    p.add_argument("--shapes", default="",
                   help="JSON {section: {precision: [tile_rows, fwd_steps, adj_steps]}} of "
                        "fixed launch shapes (no autotuning), e.g. from a previous line's "
                        "launch_shape entries")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a 256 MiB device copy (counter calibration)")
    return p.parse_args(argv)


def ev():
    import torch
    e = torch.cuda.Event(enable_timing=True)
    e.record()
    return e


def rel(a, b):
    import numpy as np
    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def kernel_name(sweep, dtype, thermal, ty, spl):
    base = "lks_step" if sweep == "fwd" else "alks_step"
    k = base + ("2_kernel" if spl == 2 else "_kernel")
    return f"{k}<{dtype}, {'true' if thermal else 'false'}, {ty}>"


def sources_sha():
    return {f: hashlib.sha256(open(os.path.join(CSRC, f), "rb").read()).hexdigest()
            for f in KERNEL_SOURCES}


def traffic_per_launch(section, kernel):
    """HBM bytes per launch of `kernel` in bench section `section` from the
    committed rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE in KiB per
    dispatch, each scaled by its reading for a plain copy of known size), or
    None when the summary was taken on other kernel sources or lacks it."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    k = t.get("entries", {}).get(f"{section}|{kernel}")
    if k is None or t.get("source_sha256") != sources_sha():
        return None
    return k["fetch_kib"] * 1024 / t["fetch_factor"] + k["write_kib"] * 1024 / t["write_factor"]


def roofline(section, kernel, key, dtype, updates_per_launch, launch_us):
    """The HBM roofline entry of one kernel: algorithmic bytes (ALGO_BYTES)
    per launch over the measured launch duration, the library's bytes
    (LIB_BYTES) and the counter-measured HBM bytes beside it."""
    i = 0 if dtype == "float" else 1
    algo_b = ALGO_BYTES[key][i] * updates_per_launch
    lib_b = LIB_BYTES[key][i] * updates_per_launch
    achieved = algo_b / (launch_us * 1e-6) / 1e9
    traffic = traffic_per_launch(section, kernel)
    out = {"bound": "hbm", "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
           "avg_launch_us": launch_us, "bytes_per_node_update": ALGO_BYTES[key][i],
           "node_updates_per_launch": updates_per_launch,
           "algorithmic_bytes_per_launch": algo_b,
           "library_bytes_per_node_update": LIB_BYTES[key][i],
           "library_achieved": lib_b / (launch_us * 1e-6) / 1e9}
    if traffic is not None:
        out["hbm_measured"] = traffic / (launch_us * 1e-6) / 1e9
        out["hbm_measured_frac"] = out["hbm_measured"] / HBM_PEAK_GBS
    return out


def apply_shape(ctx, shape):
    ty, sf, sa = shape
    ctx.set_tile_rows(int(ty))
    ctx.set_steps_per_launch(int(sf), int(sa))


def shape_dict(s):
    return {"tile_rows": s[0], "forward_steps_per_launch": s[1], "adjoint_steps_per_launch": s[2]}


def steady_launch_us(ctx, g, wl, sweep, nprobe):
    """Average launch duration of the steady forward (lks_advance) or adjoint
    (alks_advance) kernel over nprobe back-to-back steps, measured with
    events on the context's stream (torch's current stream)."""
    import torch
    out = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    ctx.backward(1.0, out, 10)
    torch.cuda.synchronize()
    e0 = ev()
    if sweep == "fwd":
        ctx.advance(g, nprobe)
    else:
        ctx.adjoint_advance(1.0, nprobe, None)
    e1 = ev()
    torch.cuda.synchronize()
    ty, sf, sa = ctx.launch_shape()
    spl = sf if sweep == "fwd" else sa
    return e0.elapsed_time(e1) * 1e3 / nprobe * spl, spl


# ---------------------------------------------------------------------------
# headline: the steady 512x512 channel
# ---------------------------------------------------------------------------
def headline(args, dev, shapes):
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0,
                              n_fwd=args.n_fwd, n_adj=args.n_adj)
    nodes = wl.nx * wl.ny
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    fixed = shapes.get("headline", {})

    ctxs = {}
    for prec in ("fp32", "fp64"):
        c = lks.LKS(wl, precision=prec, device=dev)
        if prec in fixed:
            apply_shape(c, fixed[prec])
        else:
            c.autotune(g, 200)
        ctxs[prec] = c
    cm = lks.LKS(wl, precision="mixed", device=dev)
    # the FP64 forward's tile height, the FP32 adjoint's steps per launch
    apply_shape(cm, fixed.get("mixed", (ctxs["fp64"].launch_shape()[0], 1,
                                        ctxs["fp32"].launch_shape()[2])))
    ctxs["mixed"] = cm

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
        return e0.elapsed_time(e1) / k, J, out.cpu().numpy()

    res = {}
    for prec in ("fp32", "mixed", "fp64"):
        k = args.fp64_steps if prec == "fp64" else args.steps
        w = 0 if prec == "fp64" else args.warmup
        ms, J, d = timed(ctxs[prec], k, w)
        fields = {n: ctxs[prec].read(n).cpu().numpy() for n in ("drho", "ux", "uy")}
        res[prec] = {"ms": ms, "J": J, "dJ": d, "fields": fields}
    upd = nodes * (wl.n_fwd + wl.n_adj)
    ref = res["fp64"]
    paths = {}
    for prec in ("fp32", "mixed", "fp64"):
        r = res[prec]
        err = {"J": abs(r["J"] - ref["J"]) / abs(ref["J"]), "dJdgamma_l2": rel(r["dJ"], ref["dJ"]),
               "fields_l2": {n: rel(r["fields"][n], ref["fields"][n]) for n in r["fields"]}}
        ok = (max(err["fields_l2"].values()) <= BOUND_FIELDS and err["J"] <= BOUND_GRAD
              and err["dJdgamma_l2"] <= BOUND_GRAD)
        paths[prec] = {"mlups": upd / (r["ms"] * 1e-3) / 1e6, "ms_per_gradient": r["ms"],
                       "gradients_per_s": 1e3 / r["ms"], "J": r["J"],
                       "launch_shape": shape_dict(ctxs[prec].launch_shape()),
                       "vs_fp64_rel_error": err, "within_stated_error": ok}
    head = min((p for p in paths if paths[p]["within_stated_error"]),
               key=lambda p: paths[p]["ms_per_gradient"])

    # roofline of the headline path's dominant kernel: the sweep with the
    # larger share of the gradient's time
    c = ctxs[head]
    ty, sf, sa = c.launch_shape()
    fwd_us, spl_f = steady_launch_us(c, g, wl, "fwd", args.probe_steps)
    adj_us, spl_a = steady_launch_us(c, g, wl, "adj", args.probe_steps)
    fdt = "double" if head in ("fp64", "mixed") else "float"
    adt = "double" if head == "fp64" else "float"
    if wl.n_fwd / spl_f * fwd_us >= wl.n_adj / spl_a * adj_us:
        rf = roofline("headline", kernel_name("fwd", fdt, False, ty, spl_f), ("2d", "fwd"), fdt,
                      nodes * spl_f, fwd_us)
    else:
        rf = roofline("headline", kernel_name("adj", adt, False, ty, spl_a), ("2d", "adj_steady"),
                      adt, nodes * spl_a, adj_us)
    other = {"forward_launch_us": fwd_us, "adjoint_launch_us": adj_us}
    # the FP32 adjoint kernel (the FP32 and mixed paths share it)
    if head != "fp32":
        c32 = ctxs["fp32"]
        ty32, _, _ = c32.launch_shape()
        a32_us, spl32 = steady_launch_us(c32, g, wl, "adj", args.probe_steps)
        other["fp32_adjoint_roofline"] = roofline(
            "headline", kernel_name("adj", "float", False, ty32, spl32), ("2d", "adj_steady"),
            "float", nodes * spl32, a32_us)
    del ctxs, c
    torch.cuda.empty_cache()
    return {"wl": wl, "head": head, "paths": paths, "roofline": rf, "roofline_detail": other}


# ---------------------------------------------------------------------------
# further sections
# ---------------------------------------------------------------------------
def batched_bench(args, dev, shapes):
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
    if "fp32" in shapes.get("batch", {}):
        ty = int(shapes["batch"]["fp32"][0])
        b.set_tile_rows(ty)
    else:
        ty = b.autotune(gs, outs, 50)
    b.run(gs, outs, n, n)                                   # warm-up, builds the graph
    torch.cuda.synchronize()
    reps = 2
    t0 = time.perf_counter()
    for _ in range(reps):
        b.run(gs, outs, n, n)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / reps
    # the batched ALKS step alone (no forward steps), then the LKS step alone
    b.run(gs, outs, 0, n)
    torch.cuda.synchronize()
    e0 = ev()
    b.run(gs, outs, 0, n)
    e1 = ev()
    torch.cuda.synchronize()
    adj_us = e0.elapsed_time(e1) * 1e3 / n
    # a run needs one adjoint step: n forward steps and one adjoint step
    b.run(gs, outs, n, 1)
    torch.cuda.synchronize()
    e0 = ev()
    b.run(gs, outs, n, 1)
    e1 = ev()
    torch.cuda.synchronize()
    fwd_us = (e0.elapsed_time(e1) * 1e3 - adj_us) / n
    return {"designs": 64, "nodes": nodes, "n_fwd": n, "n_adj": n, "ms_per_batch": ms,
            "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
            "gradients_per_s": 64 * 1e3 / ms, "launch_shape": shape_dict((ty, 1, 1)),
            "roofline": roofline("batch", f"alks_step_batch_kernel<float, false, {ty}>",
                                 ("2d", "adj_steady"), "float", nodes, adj_us),
            "forward_roofline": roofline("batch", f"lks_step_batch_kernel<float, false, {ty}>",
                                         ("2d", "fwd"), "float", nodes, fwd_us)}


def ubatch_bench(args, dev, shapes):
    """64 independent unsteady forced-convection designs (edge lengths from
    {128,...,512}, Re in [10, 200], Pr = 6, oscillating inflow, time-averaged
    enthalpy flux through the last interior column) over one horizon of n
    steps: the forward sweep and the checkpointed adjoint sweep of all
    designs, one launch per step for all of them, replayed as a HIP graph;
    one checkpoint interval for the batch from its memory budget (16 GiB
    FP32, 32 GiB FP64).

    Step times: a forward-only run (n_adj = 0) gives the LKS step; a full
    run takes n + R LKS steps (R replayed) and n + 1 ALKS steps."""
    import numpy as np
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.ubatch_steps
    wls = W.batch_unsteady_designs(64, n_steps=n)
    nodes = sum(w.nx * w.ny for w in wls)
    gs = [torch.tensor(w.gamma.reshape(-1), dtype=torch.float64, device=dev) for w in wls]

    def timed(prec, budget, ty, reps=2, steps=False):
        b = lks.Batch(wls, precision=prec, device=dev, mem_budget=budget)
        b.set_tile_rows(ty)
        outs = [torch.empty_like(x) for x in gs]
        Js = b.run(gs, outs, n, n)                      # warm-up, builds the graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            b.run(gs, outs, n, n)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        K, rep, ws = b.checkpoint_info()
        out = {"ms_per_batch": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
               "gradients_per_s": 64 * 1e3 / ms, "K": K, "replay_steps": rep,
               "workspace_GiB": ws / 2 ** 30, "budget_GiB": budget / 2 ** 30, "tile_rows": ty}
        sens = np.concatenate([o.cpu().numpy() for o in outs])
        if steps:
            b.run(gs, outs, n, 0)                       # forward-only graph
            torch.cuda.synchronize()
            e0 = ev()
            b.run(gs, outs, n, 0)
            e1 = ev()
            b.run(gs, outs, n, n)
            e2 = ev()
            torch.cuda.synchronize()
            fwd_us = e0.elapsed_time(e1) * 1e3 / n
            adj_us = (e1.elapsed_time(e2) * 1e3 - (n + rep) * fwd_us) / (n + 1)
            out.update({"forward_step_us": fwd_us, "adjoint_step_us": adj_us})
        b.close()
        del b, outs
        torch.cuda.empty_cache()
        return out, np.array(Js), sens

    res = {"designs": 64, "nodes": nodes, "steps": n}
    sh = shapes.get("ubatch", {})
    ty32 = int(sh["fp32"][0]) if "fp32" in sh else None
    if ty32 is None:                                    # the faster tile height
        tries = {ty: timed("fp32", 16 * 2 ** 30, ty, reps=1)[0]["ms_per_batch"] for ty in (4, 8)}
        ty32 = min(tries, key=tries.get)
    a, J32, s32 = timed("fp32", 16 * 2 ** 30, ty32, steps=True)
    ty64 = int(sh["fp64"][0]) if "fp64" in sh else 8
    c, J64, s64 = timed("fp64", 32 * 2 ** 30, ty64)
    res.update({"fp32": a, "fp64": c,
                "speedup_fp32_vs_fp64": c["ms_per_batch"] / a["ms_per_batch"],
                "fp32_vs_fp64_rel_error": {
                    "J_max": float(np.max(np.abs(J32 - J64) / np.abs(J64))),
                    "dJdgamma_l2": rel(s32, s64)}})
    res["roofline"] = roofline("ubatch", f"alks_step_ubatch_kernel<float, true, {ty32}>",
                               ("2d_thermal", "adj_unsteady"), "float", nodes,
                               a["adjoint_step_us"])
    res["roofline"]["note"] = ("step duration: the full run less its forward and replayed "
                               "steps at the forward-only run's step time")
    res["forward_roofline"] = roofline("ubatch", f"lks_step_ubatch_kernel<float, true, {ty32}>",
                                       ("2d_thermal", "fwd"), "float", nodes,
                                       a["forward_step_us"])
    return res


def large_bench(args, dev, shapes):
    """The headline's steady channel at 2048x2048 (Re = 100, the same gamma
    recipe), n + n steps in FP32: enough tiles to fill the chip, so the
    kernels are measured against HBM bandwidth rather than launch latency."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.large_steps
    wl = W.steady_channel_grf(2048, 2048, Re=100.0, sigma=8.0, seed=0, n_fwd=n, n_adj=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    nodes = wl.nx * wl.ny
    c = lks.LKS(wl, precision="fp32", device=dev)
    if "fp32" in shapes.get("large", {}):
        apply_shape(c, shapes["large"]["fp32"])
    else:
        c.autotune(g, 50)
    ty, sf, sa = c.launch_shape()
    out = torch.empty_like(g)
    torch.cuda.synchronize()
    e0 = ev()
    c.forward(g, n)
    c.objective()
    c.backward(1.0, out, n)
    e1 = ev()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    fwd_us, _ = steady_launch_us(c, g, wl, "fwd", min(args.probe_steps, 1000))
    adj_us, _ = steady_launch_us(c, g, wl, "adj", min(args.probe_steps, 1000))
    res = {"mlups": nodes * 2 * n / (ms * 1e-3) / 1e6, "ms_per_gradient": ms,
           "n_fwd": n, "n_adj": n, "nodes": nodes, "launch_shape": shape_dict((ty, sf, sa)),
           "roofline": roofline("large", kernel_name("adj", "float", False, ty, sa),
                                ("2d", "adj_steady"), "float", nodes * sa, adj_us),
           "forward_roofline": roofline("large", kernel_name("fwd", "float", False, ty, sf),
                                        ("2d", "fwd"), "float", nodes * sf, fwd_us)}
    del c
    torch.cuda.empty_cache()
    return res


def _checkpointed(ctx_fp32, ctx_fp64, g, nodes, n):
    """Time one gradient on each context; the checkpointed sweep replays
    the forward segments inside the backward call. The forward step time is
    the forward call over n; the adjoint step time is the backward call less
    the replayed steps at that forward step time, over n + 1 levels."""
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
        info = c.checkpoint_info()
        fwd_step_us = e0.elapsed_time(e1) * 1e3 / n
        adj_step_us = (e1.elapsed_time(e2) * 1e3 - info["replay_steps"] * fwd_step_us) / (n + 1)
        res[name] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                     "gradients_per_s": 1e3 / ms, "forward_ms": e0.elapsed_time(e1),
                     "backward_ms": e1.elapsed_time(e2), "K": rep["K"],
                     "replay_steps": info["replay_steps"],
                     "checkpoint_GiB": rep["ckpt_bytes"] / 2 ** 30, "J": J,
                     "forward_step_us": fwd_step_us, "adjoint_step_us": adj_step_us}
        outs[name] = out.cpu().numpy()
    res["speedup_fp32_vs_fp64"] = res["fp64"]["ms_per_gradient"] / res["fp32"]["ms_per_gradient"]
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {
        "J": abs(res["fp32"]["J"] - J64) / abs(J64) if J64 else None,
        "dJdgamma_l2": rel(outs["fp32"], outs["fp64"]) if np.any(outs["fp64"]) else None}
    return res, outs["fp32"]


def unsteady_bench(args, dev, shapes):
    """1024x512 unsteady forced convection (Re = 200, Pr = 6, oscillating
    inflow), time-averaged heat objective, 20000 steps; the adjoint replays
    the forward from checkpoints, the interval the one that fits the memory
    budget (4 GiB FP32, 8 GiB FP64) with the fewest replayed steps."""
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.unsteady_steps
    wl = W.unsteady_thermal_channel(1024, 512, n_steps=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    c32 = lks.LKS(wl, precision="fp32", mem_budget=4 * 2 ** 30, device=dev)
    c64 = lks.LKS(wl, precision="fp64", mem_budget=8 * 2 ** 30, device=dev)
    for prec, c in (("fp32", c32), ("fp64", c64)):
        if prec in shapes.get("unsteady", {}):
            apply_shape(c, shapes["unsteady"][prec])
        else:
            c.autotune(g, 100)
    nodes = wl.nx * wl.ny
    res, _ = _checkpointed(c32, c64, g, nodes, n)
    ty = c32.launch_shape()[0]
    res["launch_shape"] = {"fp32": shape_dict(c32.launch_shape()),
                           "fp64": shape_dict(c64.launch_shape())}
    res["roofline"] = roofline("unsteady", kernel_name("adj", "float", True, ty, 1),
                               ("2d_thermal", "adj_unsteady"), "float", nodes,
                               res["fp32"]["adjoint_step_us"])
    res["roofline"]["note"] = "launch duration estimated from the backward call less its replay"
    res.update({"nodes": nodes, "steps": n, "budget_GiB": {"fp32": 4, "fp64": 8}})
    del c32, c64
    torch.cuda.empty_cache()
    return res


def exchanger_bench(args, dev, shapes):
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
        if prec in shapes.get("exchanger", {}):
            apply_shape(c, shapes["exchanger"][prec])
        else:
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
                     "gradients_per_s": 1e3 / ms, "J": J,
                     "launch_shape": shape_dict(c.launch_shape())}
        outs[prec] = out.cpu().numpy()
        del c
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {"J": abs(res["fp32"]["J"] - J64) / abs(J64),
                                     "dJdgamma_l2": rel(outs["fp32"], outs["fp64"])}
    res.update({"nodes": nodes, "n_fwd": n, "n_adj": n, "beta_max": wl.beta_max})
    torch.cuda.empty_cache()
    return res


def sink_bench(args, dev, shapes):
    """Transient natural-convection heat sink 141x161 (Ra = 2e5, Pr = 6,
    K_s = 10 K_f, heat flux 0.01 on the heated boundary), mean heated
    temperature averaged over n steps, whole trajectory kept. The exact
    adjoint mode (zero thermal adjoint on prescribed-temperature walls) stays
    bounded over the horizon; the paper's form grows without bound there and
    is reported beside it. Central differences of J at four nodes (two next
    to the heated boundary, two inside) are reported with the exact-mode FP64
    gradient at those nodes."""
    import numpy as np
    import torch
    from paper_2411_03090_amd import lks, workloads as W
    n = args.sink_steps
    wl = W.heat_sink(n_steps=n)
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=dev)
    nodes = wl.nx * wl.ny
    res, outs = {}, {}
    c64 = None
    for prec, mode in (("fp32", "exact"), ("fp64", "exact"), ("fp32", "paper")):
        wl.adjoint_mode = mode
        c = lks.LKS(wl, precision=prec, device=dev)
        key = prec if mode == "exact" else "fp32_paper_mode"
        if key in shapes.get("sink", {}):
            apply_shape(c, shapes["sink"][key])
        else:
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
        res[key] = {"ms_per_gradient": ms, "mlups": nodes * 2 * n / (ms * 1e-3) / 1e6,
                    "gradients_per_s": 1e3 / ms, "J": J,
                    "launch_shape": shape_dict(c.launch_shape()),
                    "dJdgamma_finite": bool(np.isfinite(o).all()),
                    "dJdgamma_max_abs": float(np.abs(o).max()) if np.isfinite(o).all() else None}
        outs[key] = o
        if key == "fp64":
            c64 = c
        else:
            del c
    J64 = res["fp64"]["J"]
    res["fp32_vs_fp64_rel_error"] = {"J": abs(res["fp32"]["J"] - J64) / abs(J64),
                                     "dJdgamma_l2": rel(outs["fp32"], outs["fp64"])}
    # central differences of J (FP64 forward runs) at sampled nodes
    eps = 1e-3
    pts = [(1, 70), (2, 70), (61, 55), (120, 40)]
    fd = []
    base = wl.gamma.copy()
    for (j, i) in pts:
        vals = []
        for e in (eps, -eps):
            gg = base.copy()
            gg[j, i] += e
            c64.forward(torch.tensor(gg.reshape(-1), dtype=torch.float64, device=dev))
            vals.append(c64.objective())
        fd.append({"node": [i, j], "fd": (vals[0] - vals[1]) / (2 * eps),
                   "alks_exact_fp64": float(outs["fp64"].reshape(wl.ny, wl.nx)[j, i])})
    res["fd_check_eps_1e-3"] = fd
    res.update({"nodes": nodes, "steps": n, "adjoint_mode": "exact"})
    del c64
    torch.cuda.empty_cache()
    return res


def duct3d_bench(args, dev, shapes):
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
    res["roofline"] = roofline("duct3d", "alks3_face_kernel + alks3f_kernel + alks3e_kernel"
                               "<float, true> (one fused ALKS step)",
                               ("3d_thermal", "adj_unsteady"), "float", nodes,
                               res["fp32"]["adjoint_step_us"])
    res["roofline"]["note"] = "step duration estimated from the backward call less its replay"
    res["forward_roofline"] = roofline("duct3d", "lks3z_kernel + copy3_kernel<float, true> "
                                       "(one LKS step)", ("3d_thermal", "fwd"), "float", nodes,
                                       res["fp32"]["forward_step_us"])
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


DTYPES = {"fp32": "f32", "fp64": "f64", "mixed": "f64 forward, f32 adjoint"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the path is a single-GPU kernel sweep and no "
              "multi-GPU figure is produced", file=sys.stderr)
        sys.exit(2)

    import torch

    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
        return
    only = set(s for s in args.only.split(",") if s) or set(SECTIONS)
    unknown = only - set(SECTIONS)
    if unknown:
        print(f"unknown sections {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)
    shapes = json.loads(args.shapes) if args.shapes else {}
    skip = {"batch": args.no_batch, "ubatch": args.no_ubatch, "large": args.no_large,
            "unsteady": args.no_unsteady,
            "exchanger": args.no_exchanger, "sink": args.no_sink, "duct3d": args.no_3d}
    run = {s: (s in only and not skip.get(s, False)) for s in SECTIONS}

    line = {"metric": "MLUPS forward+adjoint and design gradients/sec vs plain FP64 GPU at "
                      "stated error"}
    if run["headline"]:
        h = headline(args, dev, shapes)
        wl, head, paths = h["wl"], h["head"], h["paths"]
        p = paths[head]
        line.update({
            "value": p["mlups"], "unit": "MLUPS", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": p["ms_per_gradient"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": DTYPES[head], "data": "synthetic",
            "config": {"workload": "steady channel 512x512 D2Q9, Re=100, gamma smoothed "
                                   "Gaussian field (sigma=8), pressure-drop objective, one "
                                   "gradient",
                       "nx": wl.nx, "ny": wl.ny, "n_fwd": wl.n_fwd, "n_adj": wl.n_adj,
                       "headline_path": head,
                       "stated_error_bounds": {"fields_l2": BOUND_FIELDS, "J": BOUND_GRAD,
                                               "dJdgamma_l2": BOUND_GRAD}},
            "gradients_per_s": p["gradients_per_s"],
            "paths": paths,
            "speedup_vs_fp64_gpu": paths["fp64"]["ms_per_gradient"] / p["ms_per_gradient"],
            "roofline": h["roofline"],
            "roofline_detail": h["roofline_detail"]})
        if not args.no_cpu_baseline:
            line["cpu_baseline"] = cpu_baseline(wl, args.cpu_sample_steps)
    for name, key, fn in (("batch", "batched_64_designs", batched_bench),
                          ("ubatch", "batched_64_unsteady_thermal_designs", ubatch_bench),
                          ("large", "steady_2048x2048", large_bench),
                          ("unsteady", "unsteady_thermal_1024x512", unsteady_bench),
                          ("exchanger", "heat_exchanger_201x201", exchanger_bench),
                          ("sink", "heat_sink_141x161", sink_bench),
                          ("duct3d", "duct3d_256x128x128", duct3d_bench)):
        line[key] = fn(args, dev, shapes) if run[name] else None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
