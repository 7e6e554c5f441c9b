"""GPU parity with the Boussinesq force G = g beta (T - T_ref) switched on
(D2Q9): forward and adjoint single steps from random states in both adjoint
modes, whole unsteady gradients against the oracle, and the closed form of a
uniformly forced box."""
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
GB = (0.003, -0.02)


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


def _channel(mode="paper"):
    wl = W.unsteady_thermal_channel(96, 21, Re=50.0, sigma=3.0, seed=3, n_steps=1)
    wl.mode, wl.ufac = W.MODE_STEADY, np.ones(2)
    wl.gbeta, wl.T_ref, wl.adjoint_mode = GB, 0.4, mode
    return wl


def _box(mode="paper"):
    wl = W.periodic_box(40, 21, nu=0.08, thermal=True)
    wl.alpha_max, wl.Ks_over_Kf, wl.objective = 0.7, 3.0, W.OBJ_HEAT
    wl.gamma = np.clip(W.gamma_grf(40, 21, 2.0, 5), 0.05, 1.0)
    wl.mask = wl.mask.copy()
    wl.mask[2:5, 3] |= W.TAG_PROBE
    wl.gbeta, wl.T_ref, wl.adjoint_mode = GB, 0.4, mode
    return wl


CASES = {"channel_96x21": _channel, "box_40x21": _box}


def _state(wl, rng):
    N = wl.nx * wl.ny
    return O.State(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(N),
                   0.02 * rng.standard_normal(N), rng.random(N))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_forward_step_with_force(case, prec):
    say(f"[gpu] Boussinesq forward step {case} {prec}")
    wl = CASES[case]()
    rng = np.random.default_rng(21)
    s = _state(wl, rng)
    pb = O.Problem(wl)
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    want = O.lks_step(pb, a, B, float(wl.ufac[min(1, len(wl.ufac) - 1)]), s)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    for n in ("drho", "ux", "uy", "T"):
        ctx.write(n, T(getattr(s, n)))
    ctx.advance(g, 1)
    tol = 1e-13 if prec == "fp64" else 1e-5
    for n in ("drho", "ux", "uy", "T"):
        assert rel(ctx.read(n).cpu().numpy(), getattr(want, n)) < tol, n


@pytest.mark.parametrize("mode", ["paper", "exact"])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_adjoint_step_with_force(case, prec, mode):
    say(f"[gpu] Boussinesq adjoint step {case} {prec} {mode}")
    wl = CASES[case](mode)
    rng = np.random.default_rng(22)
    s = _state(wl, rng)
    N = wl.nx * wl.ny
    pb = O.Problem(wl)
    a, da, B, dB = O.coefficients(pb, wl.gamma)
    prop = a if mode == "exact" else None
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx1, Vy1, Th1 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj1, alpha=prop)
    seed = 0.5
    sdp = seed if wl.objective == W.OBJ_PRESSURE_DROP else 0.0
    sh = seed if wl.objective == W.OBJ_HEAT else 0.0
    adj0 = O.alks_step(pb, a, B, s, s, adj1, sdp, sh)
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
def test_unsteady_gradient_with_force(mode):
    say(f"[gpu] Boussinesq unsteady thermal 70x26 160 steps fp64 {mode}")
    wl = W.unsteady_thermal_channel(70, 26, Re=60.0, sigma=3.0, seed=4, n_steps=160,
                                    period=80.0)
    wl.gbeta, wl.T_ref, wl.adjoint_mode = (0.0, 0.004), 0.5, mode
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
    """A uniform state under a uniform force: u_n = u_inf + (u_0 - u_inf)
    (1 + alpha)^-n with u_inf = G / alpha (the uniform-box pin of the
    oracle), here through the GPU steady sweep."""
    say("[gpu] Boussinesq uniform box closed form")
    nx, ny, a0 = 24, 10, 0.3
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.alpha_max, wl.q_alpha = a0 * 1.1, 0.1  # alpha at gamma: a0 (set below)
    wl.gbeta, wl.T_ref = GB, 0.25
    # gamma giving alpha = a0 everywhere: alpha = amax q (1-g)/(q+g)
    q, amax = wl.q_alpha, wl.alpha_max
    gam = q * (amax - a0) / (a0 + amax * q)
    wl.gamma = np.full((ny, nx), gam)
    ctx = lks.LKS(wl, precision="fp64", device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    N = nx * ny
    T0, u0 = 0.8, np.array([0.01, -0.02])
    ctx.write("drho", T(np.zeros(N)))
    ctx.write("ux", T(np.full(N, u0[0])))
    ctx.write("uy", T(np.full(N, u0[1])))
    ctx.write("T", T(np.full(N, T0)))
    n = 30
    ctx.advance(g, n)
    G = np.array(GB) * (T0 - 0.25)
    uinf = G / a0
    want = uinf + (u0 - uinf) * (1.0 + a0) ** (-n)
    assert np.allclose(ctx.read("ux").cpu().numpy(), want[0], rtol=1e-12, atol=1e-16)
    assert np.allclose(ctx.read("uy").cpu().numpy(), want[1], rtol=1e-12, atol=1e-16)
