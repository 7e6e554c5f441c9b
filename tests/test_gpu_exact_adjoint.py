"""GPU parity of the exact-discrete-adjoint mode (lks_set_adjoint_mode
LKS_ADJ_EXACT) against the oracle in the same mode: single ALKS steps from
random states, whole steady and unsteady gradients (checkpointed), D2Q9 and
D3Q19, FP64 and FP32. The propagated coefficient V is divided by 1 + alpha
in this mode, so the fields compared are the ones the library stores."""
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


def _exact(wl):
    wl.adjoint_mode = "exact"
    return wl


def _thermal_channel():
    wl = W.unsteady_thermal_channel(96, 21, Re=50.0, sigma=3.0, seed=3, n_steps=1)
    wl.mode, wl.ufac = W.MODE_STEADY, np.ones(2)
    return _exact(wl)


def _periodic_thermal(ks=1.0):
    wl = W.periodic_box(40, 21, nu=0.08, thermal=True)
    wl.alpha_max, wl.Ks_over_Kf, wl.objective = 0.7, ks, W.OBJ_HEAT
    wl.gamma = np.clip(W.gamma_grf(40, 21, 2.0, 5), 0.05, 1.0)
    wl.mask = wl.mask.copy()
    wl.mask[2:5, 3] |= W.TAG_PROBE
    return _exact(wl)


CASES2 = {
    "channel_70x37": lambda: _exact(W.steady_channel_uniform(70, 37, Re=10.0, seed=1)),
    "thermal_96x21": _thermal_channel,
    "periodic_thermal_40x21": _periodic_thermal,
    # conductivity contrast: the transposed -div_h (B q~) of the exact mode
    "periodic_contrast_40x21": lambda: _periodic_thermal(4.0),
}


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES2))
def test_exact_single_adjoint_step(case, prec):
    say(f"[gpu] exact-mode adjoint step {case} {prec}")
    wl = CASES2[case]()
    rng = np.random.default_rng(11)
    N = wl.nx * wl.ny
    s = O.State(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(N),
                0.02 * rng.standard_normal(N), rng.random(N))
    pb = O.Problem(wl)
    a, da, B, dB = O.coefficients(pb, wl.gamma)
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx1, Vy1, Th1 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj1, alpha=a)
    seed = 0.75
    sdp = seed if wl.objective == W.OBJ_PRESSURE_DROP else 0.0
    sh = seed if wl.objective == W.OBJ_HEAT else 0.0
    adj0 = O.alks_step(pb, a, B, s, s, adj1, sdp, sh)
    Vx0, Vy0, Th0 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj0, alpha=a)
    sens = np.zeros(N)
    O.sens_add(pb, a, da, dB, s, adj0, 1.0, sens)

    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    for n in ["drho", "ux", "uy"] + (["T"] if wl.thermal else []):
        ctx.write(n, T(getattr(s, n)))
    ctx.write("adj_rho", T(adj1[0]))
    ctx.write("adj_vx", T(Vx1))
    ctx.write("adj_vy", T(Vy1))
    if wl.thermal:
        ctx.write("adj_theta", T(Th1))
    dJ = torch.zeros(N, dtype=torch.float64, device=DEV)
    ctx.adjoint_advance(seed, 1, dJ)
    tol = 1e-13 if prec == "fp64" else 2e-5
    pairs = [("adj_rho", adj0[0]), ("adj_vx", Vx0), ("adj_vy", Vy0)]
    if wl.thermal:
        pairs.append(("adj_theta", Th0))
    for n, ref in pairs:
        assert rel(ctx.read(n).cpu().numpy(), ref) < tol, n
    assert rel(dJ.cpu().numpy(), sens) < tol


def _gpu_gradient(wl, prec, budget=0):
    ctx = lks.LKS(wl, precision=prec, mem_budget=budget, device=DEV)
    g = T(wl.gamma)
    dJ = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    ctx.backward(1.0, dJ, wl.n_adj)
    torch.cuda.synchronize()
    return J, dJ.cpu().numpy(), ctx


def test_exact_steady_channel_gradient_fp64():
    say("[gpu] exact mode steady channel 48x40 600+600 fp64")
    wl = _exact(W.steady_channel_uniform(48, 40, Re=10.0, seed=0, n_fwd=600, n_adj=600))
    Jo, so, _, _ = O.gradient(wl)
    J, dJ, _ = _gpu_gradient(wl, "fp64")
    assert abs(J - Jo) / abs(Jo) < 1e-12
    assert rel(dJ, so.ravel()) < 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-3)])
def test_exact_unsteady_thermal_gradient_checkpointed(prec, tol):
    say(f"[gpu] exact mode unsteady thermal 70x26 160 steps {prec}, checkpointed")
    wl = _exact(W.unsteady_thermal_channel(70, 26, Re=60.0, sigma=3.0, seed=4, n_steps=160,
                                           period=80.0))
    Jo, so, _, _ = O.gradient(wl)
    c = lks.LKS(wl, precision=prec, bind=False)
    r = 8 if prec == "fp64" else 4
    budget = (c.workspace_size() - c.memory_report()["ckpt_bytes"]
              + ((160 // 16) + 1) * 4 * wl.nx * wl.ny * r + 15 * 3 * wl.nx * wl.ny * r + 1024)
    J, dJ, ctx = _gpu_gradient(wl, prec, budget)
    assert ctx.memory_report()["K"] < 160
    assert abs(J - Jo) / abs(Jo) < (1e-12 if prec == "fp64" else 1e-4)
    assert rel(dJ, so.ravel()) < tol
    # the exact mode differs from the paper's ALKS by more than the tolerance
    wl.adjoint_mode = "paper"
    _, so_paper, _, _ = O.gradient(wl)
    assert rel(so_paper, so) > 10 * tol


@pytest.mark.parametrize("ks", [1.0, 2.0])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_exact_single_adjoint_step_3d(prec, ks):
    say(f"[gpu] exact-mode 3D adjoint step duct 18x10x12 {prec} Ks/Kf={ks}")
    wl = _exact(W.heated_block_duct(18, 10, 12, Re=20.0, Pr=0.71, sigma=2.0, seed=0, n_steps=1))
    wl.Ks_over_Kf = ks
    wl.mode, wl.ufac = W.MODE_STEADY, np.ones(2)
    rng = np.random.default_rng(12)
    pb = O3.Problem3(wl)
    N = pb.N
    s = O3.State3(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(3 * N),
                  rng.random(N))
    a, da, B, dB = O3.coefficients(pb, wl.gamma)
    adj1 = [rng.standard_normal(N) for _ in range(14)]
    V1, Th1 = O3.adjoint_equilibrium(pb, B, s.u, adj1, alpha=a)
    seed = 0.6
    sh = seed if wl.objective == W.OBJ_HEAT else 0.0
    sdp = seed if wl.objective == W.OBJ_PRESSURE_DROP else 0.0
    adj0 = O3.alks_step(pb, a, B, s, s, adj1, sdp, sh)
    V0, Th0 = O3.adjoint_equilibrium(pb, B, s.u, adj0, alpha=a)
    sens = np.zeros(N)
    O3.sens_add(pb, a, da, dB, s, adj0, 1.0, sens)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    ctx.write("drho", T(s.drho))
    for c, n in enumerate(("ux", "uy", "uz")):
        ctx.write(n, T(s.u[c * N:(c + 1) * N]))
    ctx.write("T", T(s.T))
    ctx.write("adj_rho", T(adj1[0]))
    for c, n in enumerate(("adj_vx", "adj_vy", "adj_vz")):
        ctx.write(n, T(V1[c * N:(c + 1) * N]))
    ctx.write("adj_theta", T(Th1))
    dJ = torch.zeros(N, dtype=torch.float64, device=DEV)
    ctx.adjoint_advance(seed, 1, dJ)
    tol = 1e-13 if prec == "fp64" else 3e-5
    ref = {"adj_rho": adj0[0], "adj_vx": V0[:N], "adj_vy": V0[N:2 * N], "adj_vz": V0[2 * N:],
           "adj_theta": Th0}
    for n, r in ref.items():
        assert rel(ctx.read(n).cpu().numpy(), r) < tol, n
    assert rel(dJ.cpu().numpy(), sens) < tol


@pytest.mark.parametrize("ks", [1.0, 2.0])
def test_exact_unsteady_duct_gradient_3d(ks):
    say(f"[gpu] exact mode 3D duct 18x10x12 60 steps fp64 Ks/Kf={ks}")
    wl = _exact(W.heated_block_duct(18, 10, 12, Re=20.0, Pr=0.71, sigma=2.0, seed=0, n_steps=60))
    wl.Ks_over_Kf = ks
    pb = O3.Problem3(wl)
    s, Jo, traj = O3.forward(pb, wl.gamma, wl.n_fwd, store=True)
    _, so = O3.adjoint_unsteady(pb, wl.gamma, traj, 1.0)
    ctx = lks.LKS(wl, precision="fp64", device=DEV)
    g = T(wl.gamma)
    dJ = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    ctx.backward(1.0, dJ, wl.n_fwd)
    torch.cuda.synchronize()
    assert abs(J - Jo) / abs(Jo) < 1e-12
    assert rel(dJ.cpu().numpy(), so) < 1e-12
