"""Checkpoint planning of unsteady contexts without a GPU: the scheme chosen
for a budget, the validation of lks_set_checkpointing, and the number of
forward steps the binomial reversal recomputes, checked against the least
possible count from a brute-force dynamic program over all schedules."""
import functools
import sys

import pytest

from paper_2411_03090_amd import lks, workloads as W


def _create(wl, precision="fp32", budget=0, ckpt=None):
    return lks.LKS(wl, precision=precision, mem_budget=budget, bind=False, checkpointing=ckpt)


@functools.lru_cache(None)
def least_steps(t, s):
    """Fewest LKS steps that reverse levels 0..t (each level's state handed to
    the adjoint once, in decreasing order) when level 0 is stored and s more
    states can be held: after k steps one state is stored and both parts are
    reversed recursively; without spare storage every level is recomputed
    from level 0."""
    if t == 0:
        return 0
    if s == 0:
        return t * (t + 1) // 2
    return min(k + least_steps(t - k, s - 1) + least_steps(k - 1, s) for k in range(1, t + 1))


def _thermal(n):
    return W.unsteady_thermal_channel(32, 16, n_steps=n)


def test_default_plan_is_two_level_and_reports_its_replay():
    c = _create(_thermal(100), budget=0)
    info = c.checkpoint_info()
    assert info == {"scheme": "two_level", "count": 100, "replay_steps": 0}
    store_all = c.memory_report()["ckpt_bytes"]
    base = c.workspace_size() - store_all
    c2 = _create(_thermal(100), budget=base + store_all // 2)
    i2 = c2.checkpoint_info()
    K = i2["count"]
    assert i2["scheme"] == "two_level" and 1 < K < 100
    ls = (100 // K) * K
    assert i2["replay_steps"] == ls - ls // K


@pytest.mark.parametrize("n,s", [(1, 1), (7, 0), (30, 1), (30, 2), (64, 3), (100, 4),
                                 (120, 6), (40, 40)])
def test_binomial_replay_is_the_least_possible(n, s):
    sys.setrecursionlimit(10000)
    c = _create(_thermal(n), ckpt=("binomial", s) if s else ("binomial", 0))
    info = c.checkpoint_info()
    if s == 0:
        # slots 0 means "as many as the budget holds": unlimited here
        assert info["count"] == n + 1 and info["replay_steps"] == 0
        return
    s_eff = min(s, n)
    assert info["scheme"] == "binomial" and info["count"] == s_eff + 1
    best = least_steps(n, s_eff)
    # the forward sweep itself places the first snapshots (at most n steps
    # of the schedule); the adjoint recomputes the rest
    assert best - n <= info["replay_steps"] <= best
    if s_eff >= n:
        assert info["replay_steps"] == 0


def test_binomial_plan_memory_and_workspace():
    n = 200
    N = 32 * 16
    c = _create(_thermal(n), ckpt=("binomial", 5))
    rep = c.memory_report()
    # 6 snapshots of (drho, ux, uy, T) in float
    assert rep["ckpt_bytes"] == 6 * 4 * N * 4
    assert rep["K"] == 0
    two = _create(_thermal(n))
    assert c.workspace_size() < two.workspace_size()


def test_auto_falls_back_to_binomial_below_the_two_level_minimum():
    n = 400
    c = _create(_thermal(n), ckpt=("binomial", 1))
    one_snap = 4 * 32 * 16 * 4
    base = c.workspace_size() - 2 * one_snap
    # two-level needs about 2 sqrt(n) states; give it 12
    budget = base + 12 * one_snap
    with pytest.raises(lks.LKSError) as e:
        _create(_thermal(n), budget=budget, ckpt=("two_level", 0))
    assert e.value.status == lks.LKS_E_NOMEM
    a = _create(_thermal(n), budget=budget)
    info = a.checkpoint_info()
    assert info["scheme"] == "binomial" and 2 <= info["count"] <= 12
    assert a.workspace_size() <= budget
    assert info["replay_steps"] >= n


def test_checkpointing_setter_validates():
    steady = _create(W.steady_channel_uniform(16, 12, Re=10, seed=0), "fp64")
    with pytest.raises(lks.LKSError) as e:
        steady.set_checkpointing("binomial", 2)
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    c = _create(_thermal(50))
    with pytest.raises(lks.LKSError) as e:
        lks._check(lks._lib.lks_set_checkpointing(c.ctx, 9, 0), c.ctx)
    assert e.value.status == lks.LKS_E_INVALID
    with pytest.raises(lks.LKSError) as e:
        c.set_checkpointing("two_level", 3)
    assert e.value.status == lks.LKS_E_INVALID
    with pytest.raises(lks.LKSError) as e:
        lks._check(lks._lib.lks_set_checkpointing(c.ctx, lks.LKS_CKPT_BINOMIAL, -1), c.ctx)
    assert e.value.status == lks.LKS_E_INVALID


def test_failed_replan_keeps_the_previous_plan():
    c0 = _create(_thermal(60), ckpt=("binomial", 2))
    budget = c0.workspace_size()
    c = _create(_thermal(60), budget=budget, ckpt=("binomial", 2))
    before = (c.workspace_size(), c.checkpoint_info())
    with pytest.raises(lks.LKSError) as e:
        c.set_checkpointing("binomial", 8)
    assert e.value.status == lks.LKS_E_NOMEM
    assert (c.workspace_size(), c.checkpoint_info()) == before


def test_full_size_duct_fits_four_gib_with_binomial_snapshots():
    """The 256x128x128 D3Q19 duct over 5000 steps: two-level checkpointing
    needs about 10 GB in FP32; a 4 GiB budget plans binomial snapshots and
    recomputes about two forward sweeps."""
    wl = W.heated_block_duct(256, 128, 128, n_steps=5000)
    with pytest.raises(lks.LKSError):
        _create(wl, budget=4 * 2 ** 30, ckpt=("two_level", 0))
    c = _create(wl, budget=4 * 2 ** 30)
    info = c.checkpoint_info()
    assert info["scheme"] == "binomial"
    assert c.workspace_size() <= 4 * 2 ** 30
    assert 5000 <= info["replay_steps"] <= 3 * 5000
