"""GPU: the binomial checkpoint schedule reverses the unsteady sweep exactly.
The same kernels run on the same states in every scheme, so J and dJ/dgamma
must be bitwise those of the stored trajectory (and of the oracle within
FP64 rounding), for any number of snapshots, in D2Q9 and D3Q19."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from paper_2411_03090_amd import lks, workloads as W  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device=DEV)


def _run(wl, prec, ckpt, budget=0):
    ctx = lks.LKS(wl, precision=prec, mem_budget=budget, device=DEV, checkpointing=ckpt)
    g = T(wl.gamma)
    dJ = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    Tn = ctx.read("T").cpu().numpy()
    ctx.backward(1.0, dJ, wl.n_fwd)
    torch.cuda.synchronize()
    return J, dJ.cpu().numpy(), Tn, ctx.checkpoint_info()


def _thermal(mode="paper"):
    wl = W.unsteady_thermal_channel(70, 26, Re=60.0, sigma=3.0, seed=4, n_steps=97,
                                    period=40.0)
    wl.adjoint_mode = mode
    return wl


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_binomial_gradient_is_bitwise_the_stored_trajectory_2d(prec):
    wl = _thermal()
    say(f"[gpu] binomial checkpointing 70x26 97 steps {prec}: store-all reference")
    J0, d0, T0, i0 = _run(wl, prec, ("two_level", 0))
    assert i0["count"] == 97 and i0["replay_steps"] == 0
    for s in (1, 2, 5, 13):
        say(f"[gpu] binomial checkpointing {prec} with {s} snapshots")
        J, d, Tn, info = _run(wl, prec, ("binomial", s))
        assert info["scheme"] == "binomial" and info["count"] == s + 1
        assert J == J0
        assert np.array_equal(Tn, T0)
        assert np.array_equal(d, d0), s
    if prec == "fp64":
        Jo, so, _, _ = O.gradient(wl)
        assert abs(J0 - Jo) / abs(Jo) < 1e-12
        assert np.linalg.norm(d0 - so.ravel()) / np.linalg.norm(so) < 1e-12


def test_binomial_without_spare_snapshots_and_exact_mode():
    """No snapshot besides level 0 (every level recomputed from the start),
    in exact mode (no level-0 sensitivity) with the heat source on."""
    wl = W.unsteady_thermal_channel(70, 26, Re=60.0, sigma=3.0, seed=4, n_steps=23,
                                    period=40.0)
    wl.adjoint_mode, wl.beta_max, wl.objective = "exact", 0.1, W.OBJ_HEAT_EXCHANGE
    say("[gpu] binomial checkpointing, level 0 only, 23 steps, exact mode")
    J0, d0, _, _ = _run(wl, "fp64", ("two_level", 0))
    # one byte below the plan with one spare snapshot
    c = lks.LKS(wl, precision="fp64", mem_budget=0, bind=False,
                checkpointing=("binomial", 1))
    budget = c.workspace_size() - 1
    c.close()
    J, d, _, info = _run(wl, "fp64", ("binomial", 0), budget=budget)
    assert info["count"] == 1 and info["replay_steps"] == 23 * 24 // 2
    assert J == J0 and np.array_equal(d, d0)


def test_two_level_segments_agree_with_binomial():
    wl = _thermal()
    say("[gpu] two-level K=10 against binomial 3 snapshots, fp32")
    c = lks.LKS(wl, precision="fp32", bind=False)
    store_all = c.memory_report()["ckpt_bytes"]
    base = c.workspace_size() - store_all
    c.close()
    J2, d2, _, i2 = _run(wl, "fp32", ("two_level", 0), budget=base + store_all // 4)
    assert i2["scheme"] == "two_level" and i2["replay_steps"] > 0
    J3, d3, _, _ = _run(wl, "fp32", ("binomial", 3))
    assert J2 == J3 and np.array_equal(d2, d3)


def test_binomial_gradient_is_bitwise_the_stored_trajectory_3d():
    wl = W.heated_block_duct(40, 18, 14, Re=30.0, sigma=3.0, seed=2, n_steps=41)
    say("[gpu] binomial checkpointing D3Q19 40x18x14 41 steps fp32")
    J0, d0, _, _ = _run(wl, "fp32", ("two_level", 0))
    J, d, _, info = _run(wl, "fp32", ("binomial", 4))
    assert info["scheme"] == "binomial" and info["replay_steps"] > 0
    assert J == J0 and np.array_equal(d, d0)
