"""GPU parity with prescribed heat flux (qbar != 0) and the heat-sink
objective (D2Q9; the D3Q19 face closure too): forward steps, adjoint steps
with the boundary seed on heated nodes (u.n = 0 walls and a u.n != 0 outlet),
unsteady heat-sink gradients in both adjoint modes, and the one-step flux
balance from rest."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import oracle as O  # noqa: E402
from oracle import d3 as O3  # noqa: E402
from paper_2411_03090_amd import lks, workloads as W  # noqa: E402

DEV = torch.device("cuda:0")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.ascontiguousarray(a, dtype=np.float64).reshape(-1), device=DEV)


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _sink(mode="paper"):
    """131 x 131 cavity (three 64-wide tiles, the last ragged)."""
    wl = W.heat_sink(n=131, Ra=2e5, q0=1e-2, Ks_over_Kf=3.0, sigma=4.0, seed=2, n_steps=1)
    wl.adjoint_mode, wl.mode, wl.ufac = mode, W.MODE_STEADY, np.ones(2)
    return wl


def _outlet(mode="paper"):
    """Thermal channel whose heated boundary is the heat-flux outlet column
    (u.n != 0 there) plus part of the adiabatic top wall, with qbar on both."""
    wl = W.unsteady_thermal_channel(96, 21, Re=50.0, sigma=3.0, seed=3, n_steps=1)
    wl.mode, wl.ufac, wl.adjoint_mode = W.MODE_STEADY, np.ones(2), mode
    wl.objective = W.OBJ_HEAT_SINK
    m = wl.mask.copy() & ~np.uint8(W.TAG_PROBE)
    m[2:-2, -1] |= W.TAG_PROBE
    m[-1, 40:70] |= W.TAG_PROBE
    wl.mask = m
    wl.Tbar = wl.Tbar.copy()
    wl.Tbar[1:-1, -1] = 0.003
    wl.Tbar[-1, 40:70] = 0.01
    return wl


CASES = {"sink_131": _sink, "outlet_96x21": _outlet}


def _state(wl, rng):
    N = wl.nx * wl.ny
    return O.State(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(N),
                   0.02 * rng.standard_normal(N), rng.random(N))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_forward_step_with_heat_flux(case, prec):
    say(f"[gpu] heat flux forward step {case} {prec}")
    wl = CASES[case]()
    rng = np.random.default_rng(41)
    s = _state(wl, rng)
    pb = O.Problem(wl)
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    want = O.lks_step(pb, a, B, float(wl.ufac[1]), s)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    for n in ("drho", "ux", "uy", "T"):
        ctx.write(n, T(getattr(s, n)))
    ctx.advance(g, 1)
    tol = 1e-13 if prec == "fp64" else 1e-5
    for n in ("drho", "ux", "uy", "T"):
        assert rel(ctx.read(n).cpu().numpy(), getattr(want, n)) < tol, n
    assert ctx.objective() == pytest.approx(O.level_objective(pb, want),
                                            rel=1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("mode", ["paper", "exact"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_step_with_boundary_seed(case, prec, mode):
    say(f"[gpu] heat-sink adjoint step {case} {prec} {mode}")
    wl = CASES[case](mode)
    rng = np.random.default_rng(42)
    s = _state(wl, rng)
    N = wl.nx * wl.ny
    pb = O.Problem(wl)
    a, da, B, dB = O.coefficients(pb, wl.gamma)
    prop = a if mode == "exact" else None
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx1, Vy1, Th1 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj1, alpha=prop)
    seed = 0.7
    sbt = seed / O.heated_count(pb)
    adj0 = O.alks_step(pb, a, B, s, s, adj1, 0.0, 0.0, None, 0.0, sbt)
    Vx0, Vy0, Th0 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj0, alpha=prop)
    sens = np.zeros(N)
    O.sens_add(pb, a, da, dB, s, adj0, 1.0, sens)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    for n in ("drho", "ux", "uy", "T"):
        ctx.write(n, T(getattr(s, n)))
    for n, v in (("adj_rho", adj1[0]), ("adj_vx", Vx1), ("adj_vy", Vy1), ("adj_theta", Th1)):
        ctx.write(n, T(v))
    dJ = torch.zeros(N, dtype=torch.float64, device=DEV)
    ctx.adjoint_advance(seed, 1, dJ)
    tol = 1e-13 if prec == "fp64" else 2e-5
    for n, v in (("adj_rho", adj0[0]), ("adj_vx", Vx0), ("adj_vy", Vy0), ("adj_theta", Th0)):
        assert rel(ctx.read(n).cpu().numpy(), v) < tol, n
    assert rel(dJ.cpu().numpy(), sens) < tol


@pytest.mark.parametrize("mode", ["paper", "exact"])
def test_unsteady_heat_sink_gradient(mode):
    say(f"[gpu] unsteady heat sink 67x67 150 steps {mode}")
    wl = W.heat_sink(n=67, n_steps=150, Ra=1e5, Ks_over_Kf=3.0, sigma=3.0, seed=4)
    wl.adjoint_mode = mode
    Jo, so, _, _ = O.gradient(wl)
    for prec, tj, tg in (("fp64", 1e-12, 1e-12), ("fp32", 1e-5, 1e-3)):
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        g = T(wl.gamma)
        dJ = torch.empty_like(g)
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        ctx.backward(1.0, dJ, wl.n_fwd)
        torch.cuda.synchronize()
        assert abs(J - Jo) / abs(Jo) < tj, prec
        assert rel(dJ.cpu().numpy(), so) < tg, prec


def test_one_step_flux_balance_on_gpu():
    say("[gpu] heat flux one step from rest")
    wl = W.heat_sink(n=40, n_steps=10, q0=0.02, Ks_over_Kf=1.0)
    wl.gbeta = (0.0, 0.0)
    m = wl.mask.copy()
    sel = (m & 3) == W.FLOW_VELOCITY
    m[sel] = (m[sel] & 0xF3) | W.THERM_FLUX
    wl.mask, wl.mode, wl.ufac = m, W.MODE_STEADY, np.ones(2)
    ctx = lks.LKS(wl, precision="fp64", device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    N = 40 * 40
    for n, v in (("drho", 0.0), ("ux", 0.0), ("uy", 0.0), ("T", 0.4)):
        ctx.write(n, T(np.full(N, v)))
    ctx.advance(g, 1)
    Tn = ctx.read("T").cpu().numpy()
    heated = (wl.mask.ravel() & W.TAG_PROBE) != 0
    assert np.allclose(Tn[heated], 0.42, rtol=0, atol=1e-15)
    assert np.allclose(Tn[~heated], 0.4, rtol=0, atol=1e-15)


def test_d3q19_flux_faces_match_the_oracle():
    """Heated-block duct with a heat flux on part of the y = 0 wall: one
    forward step against the D3Q19 oracle."""
    say("[gpu] D3Q19 heat-flux faces, one step")
    wl = W.heated_block_duct(40, 18, 14, Re=30.0, sigma=3.0, seed=2, n_steps=1)
    wl.mode, wl.ufac = W.MODE_STEADY, np.ones(2)
    wl.Tbar = wl.Tbar.copy()
    wl.Tbar[3:10, 0, 20:30] = 0.01      # (z, y, x): y = 0 wall, adiabatic class
    pb = O3.Problem3(wl)
    a, _, B, _ = O3.coefficients(pb, wl.gamma)
    rng = np.random.default_rng(7)
    N = wl.nx * wl.ny * wl.nz
    s = O3.State3(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(3 * N),
                  rng.random(N))
    want = O3.lks_step(pb, a, B, 1.0, s)
    for prec, tol in (("fp64", 1e-13), ("fp32", 1e-5)):
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        g = T(wl.gamma)
        ctx.forward(g, 0)
        ctx.write("drho", T(s.drho))
        ctx.write("ux", T(s.u[:N]))
        ctx.write("uy", T(s.u[N:2 * N]))
        ctx.write("uz", T(s.u[2 * N:]))
        ctx.write("T", T(s.T))
        ctx.advance(g, 1)
        assert rel(ctx.read("T").cpu().numpy(), want.T) < tol, prec
        assert rel(ctx.read("drho").cpu().numpy(), want.drho) < tol, prec
