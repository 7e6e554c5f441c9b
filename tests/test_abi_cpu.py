"""The C-ABI library loads, exports every symbol include/lks.h declares, and
validates problems and plans memory without touching a GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2411_03090_amd import lks, workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "lks.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return set(re.findall(r"\b((?:lks|alks)_[a-z_]+)\s*\(", src))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert {"lks_create", "lks_forward", "alks_backward", "lks_objective"} <= names
    for n in sorted(names):
        assert hasattr(lks.lib(), n), n
    assert names == set(lks.EXPORTED)


def _create(wl, precision="fp64", budget=0):
    return lks.LKS(wl, precision=precision, mem_budget=budget, bind=False)


def test_create_without_gpu_and_workspace_size():
    wl = W.steady_channel_uniform(64, 64, Re=10, seed=0)
    c = _create(wl)
    n = c.workspace_size()
    # 16 state/adjoint arrays + 7 coefficient/boundary arrays of N doubles at least
    assert n >= 23 * 64 * 64 * 8
    c32 = _create(wl, "fp32")
    assert c32.workspace_size() < n
    rep = c.memory_report()
    assert rep["K"] == 0 and rep["ckpt_bytes"] == 0


@pytest.mark.parametrize("field,value,status", [
    ("nu", 0.2, lks.LKS_E_INVALID),        # A < 0
    ("nu", 0.0, lks.LKS_E_INVALID),
    ("alpha_max", -1.0, lks.LKS_E_INVALID),
    ("q_alpha", 0.0, lks.LKS_E_INVALID),
])
def test_invalid_physics_is_rejected(field, value, status):
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    setattr(wl, field, value)
    with pytest.raises(lks.LKSError) as e:
        _create(wl)
    assert e.value.status == status


def test_invalid_masks_and_inflow_are_rejected():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.mask = wl.mask.copy()
    wl.mask[0, 0] = W.FLOW_VELOCITY          # corner not classed corner
    with pytest.raises(lks.LKSError):
        _create(wl)
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.mask = wl.mask.copy()
    wl.mask[5, 5] = W.FLOW_VELOCITY          # interior node with a boundary class
    with pytest.raises(lks.LKSError):
        _create(wl)
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.ubar = wl.ubar * 100.0                # |u| far above the low-Mach limit
    with pytest.raises(lks.LKSError):
        _create(wl)
    wl = W.unsteady_thermal_channel(16, 12, n_steps=10)
    wl.nu, wl.Pr = 0.1, 0.5                  # K_f = 0.2 > 1/6 gives B < 0
    with pytest.raises(lks.LKSError) as e:
        _create(wl)
    assert "B < 0" in str(e.value)


def test_heat_objective_needs_thermal():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.objective = W.OBJ_HEAT
    with pytest.raises(lks.LKSError):
        _create(wl)


def test_boussinesq_force_needs_a_thermal_d2q9_problem():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.gbeta = (0.0, 0.01)
    with pytest.raises(lks.LKSError) as e:
        _create(wl)
    assert e.value.status == lks.LKS_E_INVALID
    wl3 = W.heated_block_duct(16, 8, 8, Re=20.0, n_steps=10)
    wl3.gbeta = (0.0, 0.01, 0.0)
    with pytest.raises(lks.LKSError) as e:
        _create(wl3)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    wt = W.unsteady_thermal_channel(16, 12, n_steps=10)
    wt.gbeta, wt.T_ref = (0.0, 0.01), 0.5
    _create(wt)


def test_heat_source_validation_and_workspace():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    wl.beta_max = 0.1
    with pytest.raises(lks.LKSError) as e:          # needs a thermal problem
        _create(wl)
    assert e.value.status == lks.LKS_E_INVALID
    wx = W.heat_exchanger(n=16, Re=10.0, n_fwd=10, n_adj=10)
    base = _create(wx).workspace_size()
    for field, value in (("beta_max", -0.1), ("beta_max", float("nan")), ("q_beta", 0.0)):
        w = W.heat_exchanger(n=16, Re=10.0, n_fwd=10, n_adj=10)
        setattr(w, field, value)
        with pytest.raises(lks.LKSError) as e:
            _create(w)
        assert e.value.status == lks.LKS_E_INVALID, field
    w = W.heat_exchanger(n=16, Re=10.0, n_fwd=10, n_adj=10)
    w.beta_max = 0.0                                  # objective without a source
    with pytest.raises(lks.LKSError) as e:
        _create(w)
    assert e.value.status == lks.LKS_E_INVALID
    w.objective = W.OBJ_PRESSURE_DROP
    # the source adds beta and beta' (two arrays of N doubles)
    assert base - _create(w).workspace_size() == 2 * 16 * 16 * 8
    wl3 = W.heated_block_duct(16, 8, 8, Re=20.0, n_steps=10)
    wl3.beta_max = 0.1
    with pytest.raises(lks.LKSError) as e:
        _create(wl3)
    assert e.value.status == lks.LKS_E_UNSUPPORTED


def test_heat_sink_objective_validation():
    _create(W.heat_sink(n=16, n_steps=10))
    w = W.heat_sink(n=16, n_steps=10)
    w.mask = w.mask.copy()
    w.mask[5, 5] |= W.TAG_PROBE                      # interior heated node
    with pytest.raises(lks.LKSError) as e:
        _create(w)
    assert e.value.status == lks.LKS_E_INVALID
    w = W.heat_sink(n=16, n_steps=10)
    w.mask = w.mask.copy()
    w.mask[3, 0] |= W.TAG_PROBE                      # prescribed-temperature wall
    with pytest.raises(lks.LKSError) as e:
        _create(w)
    assert e.value.status == lks.LKS_E_INVALID
    w = W.heat_sink(n=16, n_steps=10)
    w.mask = w.mask & ~np.uint8(W.TAG_PROBE)         # no heated node
    with pytest.raises(lks.LKSError) as e:
        _create(w)
    assert e.value.status == lks.LKS_E_INVALID
    w = W.heat_sink(n=16, n_steps=10)
    w.Tbar = w.Tbar.copy()
    w.Tbar[0, 3] = np.inf
    with pytest.raises(lks.LKSError) as e:
        _create(w)
    assert e.value.status == lks.LKS_E_INVALID
    w3 = W.heated_block_duct(16, 8, 8, Re=20.0, n_steps=10)
    w3.objective = W.OBJ_HEAT_SINK
    with pytest.raises(lks.LKSError) as e:
        _create(w3)
    assert e.value.status == lks.LKS_E_UNSUPPORTED


def test_adjoint_mode_setter_validates():
    c = _create(W.steady_channel_uniform(16, 12, Re=10, seed=0))
    c.set_adjoint_mode("exact")
    c.set_adjoint_mode("paper")
    with pytest.raises(lks.LKSError) as e:
        lks._check(lks._lib.lks_set_adjoint_mode(c.ctx, 7), c.ctx)
    assert e.value.status == lks.LKS_E_INVALID


def test_d3q19_duct_validates_and_plans_without_gpu():
    wl = W.heated_block_duct(32, 16, 12, Re=50.0, n_steps=100)
    c = _create(wl, "fp32")
    N = 32 * 16 * 12
    rep = c.memory_report()
    assert rep["K"] == 100                       # whole trajectory kept
    # level-0 checkpoint (drho, u, T) plus 100 levels of (u, T)
    assert rep["ckpt_bytes"] == (5 + 100 * 4) * N * 4
    # the full-size heated-block duct: 5000 levels do not fit 288 GB whole
    big = W.heated_block_duct(256, 128, 128, n_steps=5000)
    Nb = 256 * 128 * 128
    full = _create(big, "fp32")
    assert full.memory_report()["ckpt_bytes"] == (5 + 5000 * 4) * Nb * 4
    assert full.memory_report()["ckpt_bytes"] > 288 * 2 ** 30
    cb = _create(big, "fp32", 16 * 2 ** 30)
    r = cb.memory_report()
    assert 1 < r["K"] < 5000 and cb.workspace_size() <= 16 * 2 ** 30


def _expect_invalid(wl):
    with pytest.raises(lks.LKSError) as e:
        _create(wl)
    assert e.value.status == lks.LKS_E_INVALID


def test_invalid_d3q19_masks_are_rejected():
    base = lambda: W.heated_block_duct(20, 10, 8, Re=20.0, n_steps=10)
    wl = base()
    wl.mask = wl.mask.copy()
    wl.mask[0, 0, 5] = W.FLOW_VELOCITY            # edge node not classed copy
    _expect_invalid(wl)
    wl = base()
    wl.mask = wl.mask.copy()
    wl.mask[3, 4, 0] = W.THERM_DIRICHLET          # face node without a flow class
    _expect_invalid(wl)
    wl = base()
    wl.mask = wl.mask.copy()
    wl.mask[3, 0, 6] |= W.TAG_SOLID               # SOLID on a face node
    _expect_invalid(wl)
    wl = base()
    wl.periodic_axes = 9
    _expect_invalid(wl)
    wl = base()
    wl.mask = wl.mask.copy()
    wl.mask[3, 4, 5] |= W.TAG_J_INLET             # pressure-drop tag inside
    _expect_invalid(wl)


def test_launch_shape_controls():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    c = _create(wl, "fp32")
    assert c.launch_shape() == (8, 1, 1)
    c.set_steps_per_launch(2, 1)
    c.set_tile_rows(4)
    assert c.launch_shape() == (4, 2, 1)
    with pytest.raises(lks.LKSError) as e:
        c.set_steps_per_launch(3)
    assert e.value.status == lks.LKS_E_INVALID
    # FP64: two steps per launch for the non-thermal forward sweep only
    c64 = _create(wl, "fp64")
    c64.set_steps_per_launch(2, 1)
    assert c64.launch_shape() == (8, 2, 1)
    with pytest.raises(lks.LKSError) as e:
        c64.set_steps_per_launch(1, 2)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    with pytest.raises(lks.LKSError) as e:
        _create(W.heat_exchanger(n=20, n_fwd=5, n_adj=5), "fp64").set_steps_per_launch(2, 1)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    # thermal FP32 D2Q9 problems take two steps per launch too; D3Q19 does not
    th = _create(W.heat_exchanger(n=20, n_fwd=5, n_adj=5), "fp32")
    th.set_steps_per_launch(2)
    assert th.launch_shape()[1:] == (2, 2)
    with pytest.raises(lks.LKSError) as e:
        _create(W.heated_block_duct(20, 10, 8, n_steps=5), "fp32").set_steps_per_launch(2)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    with pytest.raises(lks.LKSError) as e:
        _create(W.heated_block_duct(20, 10, 8, n_steps=5), "fp32").set_tile_rows(4)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    # unsteady sweeps: the forward (first sweep and replays) takes two steps
    # per launch; 64 x 16 tiles run one
    un = _create(W.unsteady_thermal_channel(70, 26, n_steps=9), "fp32")
    un.set_tile_rows(8)
    un.set_steps_per_launch(2, 1)
    assert un.launch_shape() == (8, 2, 1)


def test_calls_out_of_order_report_state_errors():
    wl = W.steady_channel_uniform(16, 12, Re=10, seed=0)
    c = _create(wl)
    J = ctypes.c_double()
    assert lks.lib().lks_objective(c.ctx, ctypes.byref(J)) == lks.LKS_E_STATE
    assert lks.lib().alks_backward(c.ctx, 1.0, 10, ctypes.c_void_p(8)) == lks.LKS_E_STATE
    assert lks.lib().lks_forward(c.ctx, ctypes.c_void_p(8), 10) == lks.LKS_E_STATE
    assert b"workspace" in lks.lib().lks_last_error(c.ctx)


def test_checkpoint_plan_follows_the_budget():
    wl = W.unsteady_thermal_channel(64, 32, n_steps=1000)
    N = 64 * 32
    full = _create(wl, "fp32")
    assert full.memory_report()["K"] == 1000          # whole trajectory kept
    store_all = full.memory_report()["ckpt_bytes"]
    # trajectory of 1000 levels of (u_x, u_y, T) plus the level-0 checkpoint
    assert store_all == (1000 * 3 + 4) * N * 4
    base = full.workspace_size() - store_all
    budget = base + store_all // 10
    c = _create(wl, "fp32", budget)
    rep = c.memory_report()
    assert 1 < rep["K"] < 1000
    assert c.workspace_size() <= budget
    # the plan replays the fewest steps of all the intervals that fit
    K = rep["K"]

    def replay(k):
        ls = (1000 // k) * k
        return 0 if k > 1000 else ls - ls // k

    def fits(k):
        return base + ((1000 // k) + 1) * 4 * N * 4 + (k - 1) * 3 * N * 4 + 2 * 256 <= budget

    assert c.checkpoint_info()["replay_steps"] == replay(K)
    assert fits(K)
    assert all(replay(k) >= replay(K) for k in range(1, 1002) if fits(k))
    with pytest.raises(lks.LKSError) as e:
        _create(wl, "fp32", base // 2)
    assert e.value.status == lks.LKS_E_NOMEM


def test_static_workspace_rejects_a_context_beyond_its_size():
    """lks_bind_static_workspace refuses, before touching the device, a
    context whose workspace exceeds the static array."""
    wl = W.steady_channel_grf(2048, 2048, Re=100.0, sigma=8.0, seed=0, n_fwd=1, n_adj=1)
    c = _create(wl, "fp32")
    assert c.workspace_size() > lks.STATIC_WORKSPACE_BYTES
    with pytest.raises(lks.LKSError) as e:
        c.bind_static()
    assert e.value.status == lks.LKS_E_NOMEM
    assert b"exceeds the static array" in lks.lib().lks_last_error(c.ctx)



def test_unsteady_batch_plans_one_interval_within_its_budget():
    """An unsteady batch validates its designs and picks one checkpoint
    interval for all of them, the one that replays the fewest steps with the
    whole batch inside the budget, without touching a GPU."""
    n = 300
    wls = W.batch_unsteady_designs(5, sizes=(24, 40, 56), n_steps=n, aspect=2)
    full = lks.Batch(wls, precision="fp32", bind=False)
    K0, rep0, ws_all = full.checkpoint_info()
    assert rep0 == 0                                   # every level kept
    # per design and interval K: 4 stored fields per checkpoint, 3 per slot
    nodes = sum(w.nx * w.ny for w in wls)

    def traj(k):
        return ((n // k) + 1) * 4 * nodes * 4 + (k - 1) * 3 * nodes * 4

    def replay(k):
        ls = (n // k) * k
        return 0 if k > n else ls - ls // k

    base = ws_all - traj(n + 1)
    budget = base + traj(n + 1) // 6
    b = lks.Batch(wls, precision="fp32", bind=False, mem_budget=budget)
    K, rep, ws = b.checkpoint_info()
    assert ws <= budget and 1 < K < n and rep == replay(K)
    slack = 2 * 256 * len(wls) * 2                     # alignment of the two arrays
    assert all(replay(k) >= rep for k in range(1, n + 2) if base + traj(k) + slack <= budget)
    # a budget no plan fits keeps the previous plan
    with pytest.raises(lks.LKSError) as e:
        b.set_memory_budget(1)
    assert e.value.status == lks.LKS_E_NOMEM
    assert b.checkpoint_info() == (K, rep, ws)
    # designs must share the horizon; batches hold no heat source
    other = W.batch_unsteady_designs(2, sizes=(24,), n_steps=n + 1)
    with pytest.raises(lks.LKSError) as e:
        lks.Batch(wls[:2] + other[:1], precision="fp32", bind=False)
    assert e.value.status == lks.LKS_E_INVALID
    hx = W.heat_exchanger(31, n_fwd=10, n_adj=10)
    with pytest.raises(lks.LKSError) as e:
        lks.Batch([hx], precision="fp32", bind=False)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
