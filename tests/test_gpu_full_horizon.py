"""Full-horizon parity: every benchmark workload at its full size and step
count on the GPU, in the launch shapes the benchmark times, against the FP64
oracle's values stored in tests/golden/full_horizon_*.json (written by
tests/golden/make_full_horizon.py, which runs the oracle alone, the unsteady
sweeps with the oracle's own two-level checkpointing).

Compared element by element at the stored seeded sample of nodes:
  FP64 GPU path  J, dJ/dgamma and the final fields to 1e-12 (relative to the
                 sample's norm, and per node relative to its largest entry);
  FP32 path      J and dJ/dgamma to 1e-3; its final fields drift with the
                 horizon (FP32 state round-off accumulated along the slow
                 modes of a developing flow) and are held to the drift the
                 benchmark reports beside the stated 1e-5 bound;
  mixed path     (FP64 forward, FP32 adjoint) fields and J to 1e-12,
                 dJ/dgamma to 1e-3.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2411_03090_amd import lks, workloads as W  # noqa: E402

DEV = torch.device("cuda:0")
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _golden(name):
    path = os.path.join(GOLDEN, f"full_horizon_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not written")
    return json.load(open(path))


def _close(got, want, tol):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    scale = np.abs(want).max()
    assert np.linalg.norm(got - want) <= tol * np.linalg.norm(want)
    assert np.all(np.abs(got - want) <= tol * scale)


def _rel(got, want):
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def _gradient(wl, precision, shape=None, budget=0):
    c = lks.LKS(wl, precision=precision, mem_budget=budget, device=DEV)
    if shape is not None:
        c.set_tile_rows(shape[0])
        c.set_steps_per_launch(shape[1], shape[2])
    g = torch.tensor(wl.gamma.reshape(-1), dtype=torch.float64, device=DEV)
    out = torch.full_like(g, float("nan"))
    c.forward(g)
    J = c.objective()
    # the final forward level, before the adjoint sweep walks back to level 0
    names = ["drho", "ux", "uy"] + (["T"] if wl.thermal else []) + \
        (["uz"] if getattr(wl, "nz", 1) > 1 else [])
    fields = {n: c.read(n).cpu().numpy() for n in names}
    c.backward(1.0, out)
    torch.cuda.synchronize()
    c.gradient_status()
    del c
    torch.cuda.empty_cache()
    return J, out.cpu().numpy(), fields


def _check(gold, J, sens, fields, tol_j, tol_g, tol_f):
    assert abs(J - gold["J"]) <= tol_j * abs(gold["J"])
    _close(sens[gold["sens_nodes"]], gold["sens"], tol_g)
    for n, want in gold["fields"].items():
        if tol_f is None:
            continue
        want = np.asarray(want)
        if not np.any(want):
            assert np.all(fields[n][gold["field_nodes"]] == 0.0), n
            continue
        _close(fields[n][gold["field_nodes"]], want, tol_f)


# the launch shapes (tile rows, forward and adjoint steps per launch) the
# benchmark's autotuner chose on an MI355X
SHAPES = {"steady_512": {"fp64": (8, 1, 1), "fp32": (8, 2, 2), "mixed": (8, 1, 2)},
          "unsteady_1024x512": {"fp64": (4, 1, 1), "fp32": (8, 1, 1)}}


@pytest.mark.parametrize("precision", ["fp64", "mixed", "fp32"])
def test_steady_512_full_horizon(precision):
    say(f"[gpu] full horizon 512x512 40000+40000 {precision}")
    gold = _golden("steady_512")
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0, n_fwd=40000, n_adj=40000)
    J, sens, fields = _gradient(wl, precision, SHAPES["steady_512"][precision])
    if precision == "fp64":
        _check(gold, J, sens, fields, 1e-12, 1e-12, 1e-12)
    elif precision == "mixed":
        _check(gold, J, sens, fields, 1e-12, 1e-3, 1e-12)
    else:
        _check(gold, J, sens, fields, 1e-3, 1e-3, None)
        drift = max(_rel(fields[n][gold["field_nodes"]], w) for n, w in gold["fields"].items())
        say(f"    fp32 field drift at 40000 steps: {drift:.2e}")
        assert drift < 5e-4


@pytest.mark.parametrize("precision,budget", [("fp64", 8 * 2 ** 30), ("fp32", 4 * 2 ** 30)])
def test_unsteady_1024x512_full_horizon(precision, budget):
    say(f"[gpu] full horizon 1024x512 unsteady thermal 20000 steps {precision}, checkpointed")
    gold = _golden("unsteady_1024x512")
    wl = W.unsteady_thermal_channel(1024, 512, n_steps=20000)
    J, sens, fields = _gradient(wl, precision, SHAPES["unsteady_1024x512"][precision], budget)
    if precision == "fp64":
        _check(gold, J, sens, fields, 1e-12, 1e-12, 1e-12)
    else:
        _check(gold, J, sens, fields, 1e-3, 1e-3, None)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32", 1e-3)])
def test_batch_64_full_horizon(precision, tol):
    say(f"[gpu] full horizon 64-design batch 2000+2000 {precision}")
    gold = _golden("batch_64")
    wls = W.batch_designs(64, n_steps=2000)
    b = lks.Batch(wls, precision=precision, device=DEV)
    if precision == "fp32":
        b.set_tile_rows(16)
    gs = [torch.tensor(w.gamma.reshape(-1), dtype=torch.float64, device=DEV) for w in wls]
    outs = [torch.full_like(x, float("nan")) for x in gs]
    Js = b.run(gs, outs, 2000, 2000)
    torch.cuda.synchronize()
    for d, (w, rec) in enumerate(zip(wls, gold["designs"])):
        assert rec["workload"] == w.name
        assert abs(Js[d] - rec["J"]) <= tol * abs(rec["J"]), d
        _close(outs[d].cpu().numpy()[rec["sens_nodes"]], rec["sens"], tol)


@pytest.mark.parametrize("precision,budget", [("fp64", 8 * 2 ** 30), ("fp32", 4 * 2 ** 30)])
def test_duct3d_full_size_200_steps(precision, budget):
    """The full-size duct over 200 steps, checkpointed, with the enthalpy-flux
    plane at x = 60, which the inflow and the block's heat reach in that time."""
    say(f"[gpu] D3Q19 duct 256x128x128, 200 steps, probe plane x = 60, {precision}, checkpointed")
    gold = _golden("duct3d_200")
    wl = W.heated_block_duct(n_steps=200, probe_col=60)
    J, sens, fields = _gradient(wl, precision, None, budget)
    assert gold["J"] > 0
    if precision == "fp64":
        _check(gold, J, sens, fields, 1e-12, 1e-12, 1e-12)
    else:
        _check(gold, J, sens, fields, 1e-3, 1e-3, 2e-5)


@pytest.mark.parametrize("precision,budget", [("fp64", 32 * 2 ** 30), ("fp32", 16 * 2 ** 30)])
def test_duct3d_full_horizon(precision, budget):
    say(f"[gpu] full horizon D3Q19 duct 256x128x128 5000 steps {precision}, checkpointed")
    gold = _golden("duct3d")
    wl = W.heated_block_duct(n_steps=5000)
    J, sens, fields = _gradient(wl, precision, None, budget)
    if precision == "fp64":
        _check(gold, J, sens, fields, 1e-12, 1e-12, 1e-12)
    else:
        _check(gold, J, sens, fields, 1e-3, 1e-3, None)
