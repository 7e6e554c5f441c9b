"""GPU parity with the heat source Q = beta_gamma (1 - T) switched on (D2Q9):
forward and adjoint single steps from random states in both adjoint modes and
with the heat-exchange objective's seed, whole steady (heat exchanger) and
unsteady gradients against the oracle, and the closed form of a uniform box."""
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


def rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def _exchanger(mode="paper", gb=(0.0, 0.0)):
    """131 x 131 (three 64-wide tiles along x, the last one ragged), mixed
    ring classes on the left and right sides."""
    wl = W.heat_exchanger(n=131, Re=20.0, beta_max=0.3, q_beta=0.2, sigma=4.0, seed=3,
                          n_fwd=1, n_adj=1)
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, gb, 0.4
    return wl


def _box(mode="paper", gb=(0.0, 0.0)):
    wl = W.periodic_box(40, 21, nu=0.08, thermal=True)
    wl.alpha_max, wl.Ks_over_Kf, wl.objective = 0.7, 3.0, W.OBJ_HEAT_EXCHANGE
    wl.beta_max, wl.q_beta = 0.25, 0.1
    wl.gamma = np.clip(W.gamma_grf(40, 21, 2.0, 5), 0.05, 1.0)
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, gb, 0.4
    return wl


CASES = {"exchanger_131": _exchanger, "box_40x21": _box}


def _state(wl, rng):
    N = wl.nx * wl.ny
    return O.State(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(N),
                   0.02 * rng.standard_normal(N), rng.random(N))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_forward_step_with_source(case, prec):
    say(f"[gpu] heat source forward step {case} {prec}")
    wl = CASES[case](gb=(0.0, 0.01))
    rng = np.random.default_rng(31)
    s = _state(wl, rng)
    pb = O.Problem(wl)
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    b, _ = O.source_coefficients(pb, wl.gamma)
    want = O.lks_step(pb, a, B, 1.0, s, b)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    for n in ("drho", "ux", "uy", "T"):
        ctx.write(n, T(getattr(s, n)))
    ctx.advance(g, 1)
    tol = 1e-13 if prec == "fp64" else 1e-5
    for n in ("drho", "ux", "uy", "T"):
        assert rel(ctx.read(n).cpu().numpy(), getattr(want, n)) < tol, n
    # the steady objective of the new level
    assert ctx.objective() == pytest.approx(O.level_objective(pb, want, b),
                                            rel=1e-12 if prec == "fp64" else 1e-5)


@pytest.mark.parametrize("gb", [(0.0, 0.0), (0.003, -0.02)])
@pytest.mark.parametrize("mode", ["paper", "exact"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_step_with_source(case, prec, mode, gb):
    say(f"[gpu] heat source adjoint step {case} {prec} {mode} gbeta={gb}")
    wl = CASES[case](mode, gb)
    rng = np.random.default_rng(32)
    s = _state(wl, rng)
    N = wl.nx * wl.ny
    pb = O.Problem(wl)
    a, da, B, dB = O.coefficients(pb, wl.gamma)
    b, db = O.source_coefficients(pb, wl.gamma)
    prop = a if mode == "exact" else None
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx1, Vy1, Th1 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj1, alpha=prop, beta=b)
    seed = 0.5
    adj0 = O.alks_step(pb, a, B, s, s, adj1, 0.0, 0.0, b, seed)
    Vx0, Vy0, Th0 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj0, alpha=prop, beta=b)
    sens = np.zeros(N)
    O.sens_add(pb, a, da, dB, s, adj0, 1.0, sens)
    O.source_sens_add(pb, a, B, b, db, s, adj0, seed, sens)
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
def test_steady_heat_exchanger_gradient(mode):
    say(f"[gpu] steady heat exchanger 70x70 500+500 steps {mode}")
    wl = W.heat_exchanger(n=70, Re=20.0, beta_max=0.2, sigma=4.0, seed=5, n_fwd=500,
                          n_adj=500)
    wl.adjoint_mode = mode
    Jo, so, _, _ = O.gradient(wl)
    for prec, tj, tg in (("fp64", 1e-12, 1e-12), ("fp32", 1e-4, 1e-3)):
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        g = T(wl.gamma)
        dJ = torch.empty_like(g)
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        ctx.backward(1.0, dJ, wl.n_adj)
        torch.cuda.synchronize()
        assert abs(J - Jo) / abs(Jo) < tj, prec
        assert rel(dJ.cpu().numpy(), so) < tg, prec


@pytest.mark.parametrize("obj", [W.OBJ_HEAT_EXCHANGE, W.OBJ_HEAT])
@pytest.mark.parametrize("mode", ["paper", "exact"])
def test_unsteady_gradient_with_source(mode, obj):
    say(f"[gpu] heat source unsteady thermal 70x26 160 steps {mode} objective {obj}")
    wl = W.unsteady_thermal_channel(70, 26, Re=60.0, sigma=3.0, seed=4, n_steps=160,
                                    period=80.0)
    wl.beta_max, wl.q_beta, wl.objective, wl.adjoint_mode = 0.15, 0.1, obj, mode
    wl.gbeta, wl.T_ref = (0.0, 0.003), 0.5
    Jo, so, _, _ = O.gradient(wl)
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-3)):
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        g = T(wl.gamma)
        dJ = torch.empty_like(g)
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        ctx.backward(1.0, dJ, wl.n_fwd)
        torch.cuda.synchronize()
        assert abs(J - Jo) / abs(Jo) < (1e-12 if prec == "fp64" else 1e-4), prec
        assert rel(dJ.cpu().numpy(), so) < tol, prec


def test_uniform_box_closed_form_on_gpu():
    """At rest with uniform T and beta: T_n = 1 - (1 - T_0)(1 + beta)^-n, and
    the heat-exchange objective of the last level is -N beta (1 - T_n)."""
    say("[gpu] heat source uniform box closed form")
    nx, ny, b0 = 24, 10, 0.2
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.objective, wl.beta_max, wl.q_beta = W.OBJ_HEAT_EXCHANGE, 0.5, 0.1
    q, bmax = wl.q_beta, wl.beta_max
    wl.gamma = np.full((ny, nx), q * (bmax - b0) / (b0 + bmax * q))
    ctx = lks.LKS(wl, precision="fp64", device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    N = nx * ny
    T0 = 0.3
    for n, v in (("drho", 0.0), ("ux", 0.0), ("uy", 0.0), ("T", T0)):
        ctx.write(n, T(np.full(N, v)))
    n = 25
    ctx.advance(g, n)
    want = 1.0 - (1.0 - T0) * (1.0 + b0) ** (-n)
    assert np.allclose(ctx.read("T").cpu().numpy(), want, rtol=1e-13, atol=0)
    assert ctx.objective() == pytest.approx(-N * b0 * (1.0 - want), rel=1e-12)
