"""Unsteady batches: many thermal designs of uneven size advanced together
through checkpointed forward and adjoint sweeps (one launch per step for all
designs, the sequence replayed as a HIP graph), against the FP64 oracle and
against each design's own context."""
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
N_STEPS = 300
_ORACLE = {}


def oracle_gradient(w, **kw):
    """The oracle's J and dJ/dgamma of a workload (cached per name and mode)."""
    key = (w.name, w.adjoint_mode)
    if key not in _ORACLE:
        J, s, _, _ = O.gradient(w, **kw)
        _ORACLE[key] = (J, s)
    return _ORACLE[key]


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device=DEV)


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def _designs(mode="paper"):
    # channels 31x31 and 40x40 (ragged tiles), one horizon over which the
    # flow reaches the probe column
    wls = W.batch_unsteady_designs(4, sizes=(24, 31, 40), sigma=3.0, n_steps=N_STEPS,
                                   periods=2.0)
    for w in wls:
        w.adjoint_mode = mode
    return wls


def _budget_batch(wls, precision, frac=0.3):
    """A batch whose budget holds the non-trajectory memory and `frac` of the
    whole trajectory (4 fields per checkpoint, 3 per replay slot)."""
    full = lks.Batch(wls, precision=precision, bind=False)
    ws_all = full.checkpoint_info()[2]
    full.close()
    r = 8 if precision == "fp64" else 4
    traj = (4 + 3 * N_STEPS) * sum(w.nx * w.ny for w in wls) * r
    return lks.Batch(wls, precision=precision, device=DEV,
                     mem_budget=int(ws_all - traj + frac * traj))


def _run(b, wls, graph=True):
    gs = [T(w.gamma) for w in wls]
    outs = [torch.full_like(g, float("nan")) for g in gs]
    Js = b.run(gs, outs, N_STEPS, N_STEPS, graph=graph)
    torch.cuda.synchronize()
    return Js, [o.cpu().numpy() for o in outs]


def _single(wl, precision, ty):
    c = lks.LKS(wl, precision=precision, device=DEV)
    c.set_tile_rows(ty)
    g = T(wl.gamma)
    d = torch.full_like(g, float("nan"))
    c.forward(g, wl.n_fwd)
    J = c.objective()
    c.backward(1.0, d)
    torch.cuda.synchronize()
    return J, d.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_unsteady_batch_matches_oracle_and_single_contexts(precision):
    say(f"[gpu] unsteady batch of 4 thermal designs, {N_STEPS} steps, {precision}")
    wls = _designs()
    b = _budget_batch(wls, precision)
    K, rep, _ = b.checkpoint_info()
    assert 1 < K <= N_STEPS and rep > 0      # checkpointed, with replay
    b.set_tile_rows(8)
    Js, sens = _run(b, wls)
    # eager launches and a second graph replay give the same bits
    Je, se = _run(b, wls, graph=False)
    Jg, sg = _run(b, wls)
    for d in range(len(wls)):
        assert Je[d] == Js[d] and Jg[d] == Js[d]
        assert np.array_equal(se[d], sens[d]) and np.array_equal(sg[d], sens[d])
    b.close()
    tol = 1e-12 if precision == "fp64" else 1e-3
    for d, w in enumerate(wls):
        # the design alone, in its own context at the same tile height
        Jc, sc = _single(w, precision, 8)
        assert Jc == Js[d], d
        assert np.array_equal(sc, sens[d]), d
        Jo, so = oracle_gradient(w, checkpoint=17)
        assert abs(Js[d] - Jo) <= tol * abs(Jo), (d, Js[d], Jo)
        assert rel(sens[d], so) <= tol, (d, rel(sens[d], so))
        say(f"    design {d} {w.name}: J={Js[d]:.6e} rel J {abs(Js[d] - Jo) / abs(Jo):.1e} "
            f"rel dJ {rel(sens[d], so):.1e}")


def test_unsteady_batch_exact_mode():
    say(f"[gpu] unsteady batch, exact adjoint mode, {N_STEPS} steps, fp64")
    wls = _designs("exact")
    b = _budget_batch(wls, "fp64", 0.25)
    b.set_tile_rows(4)
    Js, sens = _run(b, wls)
    b.close()
    for d, w in enumerate(wls):
        Jc, sc = _single(w, "fp64", 4)
        assert Jc == Js[d] and np.array_equal(sc, sens[d]), d
        Jo, so = oracle_gradient(w)
        assert abs(Js[d] - Jo) <= 1e-12 * abs(Jo)
        assert rel(sens[d], so) <= 1e-12


def test_unsteady_batch_keeps_every_level_without_a_budget():
    say(f"[gpu] unsteady batch without a budget (no replay), fp32, {N_STEPS} steps")
    wls = _designs()[:3]
    b = lks.Batch(wls, precision="fp32", device=DEV)
    K, rep, _ = b.checkpoint_info()
    assert rep == 0
    b.set_tile_rows(8)
    gs = [T(w.gamma) for w in wls]
    outs = [torch.full_like(g, float("nan")) for g in gs]
    Js = b.run(gs, outs, N_STEPS, N_STEPS)
    torch.cuda.synchronize()
    for d, w in enumerate(wls):
        Jc, sc = _single(w, "fp32", 8)
        assert Jc == Js[d] and np.array_equal(sc, outs[d].cpu().numpy()), d
        Jo, so = oracle_gradient(w)
        assert abs(Js[d] - Jo) <= 1e-3 * abs(Jo)
        assert rel(outs[d].cpu().numpy(), so) <= 1e-3
    # forward fields are not kept; adjoint fields of level 0 are
    with pytest.raises(lks.LKSError) as e:
        b.read(0, "ux")
    assert e.value.status == lks.LKS_E_UNSUPPORTED
    assert torch.isfinite(b.read(0, "adj_rho")).all()


def test_unsteady_batch_forward_only_run():
    say(f"[gpu] unsteady batch, forward sweep only (n_adj = 0), fp32, {N_STEPS} steps")
    wls = _designs()[:2]
    b = _budget_batch(wls, "fp32")
    Js, sens = _run(b, wls)
    gs = [T(w.gamma) for w in wls]
    outs = [torch.full_like(g, float("nan")) for g in gs]
    Jf = b.run(gs, outs, N_STEPS, 0)
    torch.cuda.synchronize()
    assert Jf == Js                                     # the same objectives, bitwise
    assert all(torch.isnan(o).all() for o in outs)      # no sensitivity written
    with pytest.raises(lks.LKSError) as e:
        b.read(0, "adj_rho")
    assert e.value.status == lks.LKS_E_STATE
