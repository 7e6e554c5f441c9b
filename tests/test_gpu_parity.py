"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (relative L2 over nodes, density measured as rho - 1):
FP64 path: 1e-12 for fields, objective and gradient; FP32-deviation path:
1e-5 for fields of a single step and 1e-3 for the gradient.
"""
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


def _steady_thermal(nx, ny, seed=0):
    wl = W.unsteady_thermal_channel(nx, ny, Re=50.0, sigma=3.0, seed=seed, n_steps=1)
    wl.mode = W.MODE_STEADY
    wl.ufac = np.ones(2)
    return wl


def _periodic(nx, ny, thermal):
    wl = W.periodic_box(nx, ny, nu=0.08, thermal=thermal)
    wl.alpha_max, wl.Ks_over_Kf = 0.7, 3.0
    wl.gamma = np.clip(W.gamma_grf(nx, ny, 2.0, 5), 0.05, 1.0)
    wl.mask = wl.mask.copy()
    wl.mask[2:5, 3] |= W.TAG_PROBE
    if thermal:
        wl.objective = W.OBJ_HEAT
    return wl


CASES = {
    "channel_70x37": lambda: W.steady_channel_uniform(70, 37, Re=10.0, seed=1),
    "channel_65x9": lambda: W.steady_channel_uniform(65, 9, Re=20.0, seed=2),
    "thermal_129x14": lambda: _steady_thermal(129, 14, seed=3),
    "periodic_67x13": lambda: _periodic(67, 13, False),
    "periodic_thermal_40x21": lambda: _periodic(40, 21, True),
}


def _random_state(wl, rng):
    N = wl.nx * wl.ny
    return O.State(1e-3 * rng.standard_normal(N), 0.02 * rng.standard_normal(N),
                   0.02 * rng.standard_normal(N), rng.random(N))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_single_forward_step(case, prec):
    say(f"[gpu] single forward step {case} {prec}")
    wl = CASES[case]()
    rng = np.random.default_rng(42)
    s = _random_state(wl, rng)
    pb = O.Problem(wl)
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    want = O.lks_step(pb, a, B, 1.0, s)
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    names = ["drho", "ux", "uy"] + (["T"] if wl.thermal else [])
    for n in names:
        ctx.write(n, T(getattr(s, n)))
    ctx.advance(g, 1)
    tol = 1e-13 if prec == "fp64" else 1e-5
    for n in names:
        got = ctx.read(n).cpu().numpy()
        ref = getattr(want, n)
        assert rel(got, ref) < tol, (n, rel(got, ref))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", list(CASES))
def test_single_adjoint_step(case, prec):
    say(f"[gpu] single adjoint step {case} {prec}")
    wl = CASES[case]()
    rng = np.random.default_rng(7)
    s = _random_state(wl, rng)
    pb = O.Problem(wl)
    a, da, B, dB = O.coefficients(pb, wl.gamma)
    adj1 = [rng.standard_normal(wl.nx * wl.ny) for _ in range(9)]
    Vx1, Vy1, Th1 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj1)
    seed = 0.75
    sdp = seed if wl.objective == W.OBJ_PRESSURE_DROP else 0.0
    sh = seed if wl.objective == W.OBJ_HEAT else 0.0
    adj0 = O.alks_step(pb, a, B, s, s, adj1, sdp, sh)
    Vx0, Vy0, Th0 = O.adjoint_equilibrium(pb, B, s.ux, s.uy, adj0)
    sens = np.zeros(wl.nx * wl.ny)
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
    dJ = torch.zeros(wl.nx * wl.ny, dtype=torch.float64, device=DEV)
    ctx.adjoint_advance(seed, 1, dJ)
    tol = 1e-13 if prec == "fp64" else 2e-5
    pairs = [("adj_rho", adj0[0]), ("adj_vx", Vx0), ("adj_vy", Vy0)]
    if wl.thermal:
        pairs.append(("adj_theta", Th0))
    for n, ref in pairs:
        got = ctx.read(n).cpu().numpy()
        assert rel(got, ref) < tol, (n, rel(got, ref))
    assert rel(dJ.cpu().numpy(), sens) < tol


def _gpu_gradient(wl, prec, budget=0):
    ctx = lks.LKS(wl, precision=prec, mem_budget=budget, device=DEV)
    g = T(wl.gamma)
    dJ = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    fields = {n: ctx.read(n).cpu().numpy() for n in ["drho", "ux", "uy"]}
    ctx.backward(1.0, dJ, wl.n_adj)
    torch.cuda.synchronize()
    return J, dJ.cpu().numpy().reshape(wl.ny, wl.nx), fields, ctx


@pytest.fixture(scope="module")
def channel64():
    wl = W.steady_channel_uniform(64, 64, Re=10.0, seed=0, n_fwd=3000, n_adj=3000)
    J, sens, s, adj = O.gradient(wl)
    return wl, J, sens, s


def test_steady_channel64_fp64_matches_oracle(channel64):
    say("[gpu] steady 64x64 Re=10 3000+3000 fp64")
    wl, Jo, so, st = channel64
    J, dJ, f, _ = _gpu_gradient(wl, "fp64")
    assert abs(J - Jo) / abs(Jo) < 1e-12
    assert rel(f["drho"], st.drho) < 1e-12
    assert rel(f["ux"], st.ux) < 1e-12
    assert rel(f["uy"], st.uy) < 1e-12
    assert rel(dJ, so) < 1e-12


def test_steady_channel64_fp32_within_tolerance(channel64):
    say("[gpu] steady 64x64 Re=10 3000+3000 fp32")
    wl, Jo, so, st = channel64
    J, dJ, f, _ = _gpu_gradient(wl, "fp32")
    assert abs(J - Jo) / abs(Jo) < 1e-3
    assert rel(f["ux"], st.ux) < 1e-4
    assert rel(dJ, so) < 1e-3


def test_seed_linearity_bitwise():
    say("[gpu] seed linearity")
    wl = W.steady_channel_uniform(70, 37, Re=10.0, seed=1, n_fwd=200, n_adj=100)
    ctx = lks.LKS(wl, precision="fp32", device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, wl.n_fwd)
    a = torch.empty_like(g)
    b = torch.empty_like(g)
    ctx.backward(1.0, a, wl.n_adj)
    ctx.backward(4.0, b, wl.n_adj)
    torch.cuda.synchronize()
    assert torch.equal(4.0 * a, b)


def _budget_for(wl, prec, K):
    """Workspace bytes of a plan with checkpoint interval K (thermal)."""
    c = lks.LKS(wl, precision=prec, bind=False)
    base = c.workspace_size() - c.memory_report()["ckpt_bytes"]
    r = 8 if prec == "fp64" else 4
    N = wl.nx * wl.ny
    return base + ((wl.n_fwd // K) + 1) * 4 * N * r + (K - 1) * 3 * N * r + 1024


def _unsteady(nx, ny, n):
    return W.unsteady_thermal_channel(nx, ny, Re=60.0, sigma=3.0, seed=4, n_steps=n,
                                      period=n / 2)


def test_unsteady_thermal_fp64_matches_oracle_and_checkpointing_is_exact():
    say("[gpu] unsteady thermal 70x26 240 steps fp64, store-all and checkpointed")
    wl = _unsteady(70, 26, 240)
    Jo, so, _, _ = O.gradient(wl)
    J, dJ, _, ctx = _gpu_gradient(wl, "fp64")
    assert ctx.memory_report()["K"] == 240
    assert abs(J - Jo) / abs(Jo) < 1e-12
    assert rel(dJ, so) < 1e-12
    J2, dJ2, _, ctx2 = _gpu_gradient(wl, "fp64", _budget_for(wl, "fp64", 20))
    K = ctx2.memory_report()["K"]
    assert 20 <= K < 240
    say(f"[gpu]   checkpoint interval K={K}")
    assert J2 == J
    assert np.array_equal(dJ2, dJ)


def test_unsteady_thermal_fp32_within_tolerance():
    say("[gpu] unsteady thermal 70x26 240 steps fp32 checkpointed")
    wl = _unsteady(70, 26, 240)
    Jo, so, _, _ = O.gradient(wl)
    J, dJ, _, ctx = _gpu_gradient(wl, "fp32", _budget_for(wl, "fp32", 17))
    assert ctx.memory_report()["K"] < 240
    assert abs(J - Jo) / abs(Jo) < 1e-4
    assert rel(dJ, so) < 1e-3


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32", 1e-3)])
def test_full_size_512_steady_short_run(prec, tol):
    """The 512x512 Re=100 workload at full size, in the launch configuration
    the benchmark times, over a step count the oracle finishes quickly."""
    say(f"[gpu] 512x512 Re=100 150+150 steps {prec}")
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0, n_fwd=150, n_adj=150)
    Jo, so, st, _ = O.gradient(wl)
    J, dJ, f, _ = _gpu_gradient(wl, prec)
    assert abs(J - Jo) / abs(Jo) < tol
    assert rel(f["ux"], st.ux) < (1e-12 if prec == "fp64" else 1e-5)
    assert rel(dJ, so) < tol


def test_full_size_1024x512_unsteady_thermal_short_run():
    say("[gpu] 1024x512 Re=200 Pr=6 unsteady 30 steps fp64 checkpointed")
    wl = W.unsteady_thermal_channel(1024, 512, n_steps=30, period=12.0)
    # in 30 steps from rest the flow reaches only the first columns: probe there
    wl.mask = W.channel_mask(1024, 512, thermal=True, probe_col=6)
    Jo, so, _, _ = O.gradient(wl)
    J, dJ, _, ctx = _gpu_gradient(wl, "fp64", _budget_for(wl, "fp64", 6))
    assert ctx.memory_report()["K"] < 30
    assert abs(J - Jo) / abs(Jo) < 1e-12
    assert rel(dJ, so) < 1e-12


def test_poiseuille_fixed_point_on_gpu():
    """Exact solution of the scheme at any size: the pressure-driven
    Poiseuille state is kept to round-off by the GPU step."""
    say("[gpu] poiseuille fixed point 300x130")
    nx, ny = 300, 130
    wl = W.steady_channel_uniform(nx, ny, Re=20.0, seed=0)
    wl.gamma[:] = 1.0
    H, U, nu = ny - 1, wl.u_max, wl.nu
    j = np.arange(ny)[:, None] * np.ones((1, nx))
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    ux = 4 * U * j * (H - j) / H ** 2
    drho = 24 * nu * U * (nx - 1 - i) / H ** 2
    ctx = lks.LKS(wl, precision="fp64", device=DEV)
    g = T(wl.gamma)
    ctx.forward(g, 0)
    ctx.write("drho", T(drho))
    ctx.write("ux", T(ux))
    ctx.write("uy", T(np.zeros_like(ux)))
    ctx.advance(g, 25)
    assert np.abs(ctx.read("ux").cpu().numpy() - ux.ravel()).max() < 1e-15
    assert np.abs(ctx.read("drho").cpu().numpy() - drho.ravel()).max() < 1e-15
    Jp = (ny - 2) * 8 * nu * U * (nx - 1) / H ** 2
    assert abs(ctx.objective() - Jp) / Jp < 1e-12


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_results_do_not_depend_on_tile_height(prec):
    say(f"[gpu] tile height invariance {prec}")
    wl = W.unsteady_thermal_channel(131, 37, Re=60.0, sigma=3.0, seed=2, n_steps=60, period=30.0)
    out = []
    for ty in (4, 8):
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        ctx.set_tile_rows(ty)
        g = T(wl.gamma)
        d = torch.empty_like(g)
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        ctx.backward(1.0, d)
        torch.cuda.synchronize()
        out.append((J, d.cpu().numpy()))
    assert out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["channel_70x37", "thermal_129x14", "periodic_thermal_40x21"])
def test_steps_do_not_depend_on_the_tile_height(case, prec):
    """Forward and adjoint steps from a random state are the same bit for bit
    with 64 x 4 and 64 x 8 tiles (different tile seams, halo loads and
    partial tiles)."""
    say(f"[gpu] tile-height invariance of steps {case} {prec}")
    wl = CASES[case]()
    rng = np.random.default_rng(11)
    s = _random_state(wl, rng)
    adj = [rng.standard_normal(wl.nx * wl.ny) for _ in range(4)]
    fwd = ["drho", "ux", "uy"] + (["T"] if wl.thermal else [])
    adn = ["adj_rho", "adj_vx", "adj_vy"] + (["adj_theta"] if wl.thermal else [])
    out = []
    heights = (4, 8, 16) if prec == "fp32" and not wl.thermal else (4, 8)
    for ty in heights:
        ctx = lks.LKS(wl, precision=prec, device=DEV)
        ctx.set_tile_rows(ty)
        g = T(wl.gamma)
        ctx.forward(g, 0)
        for n in fwd:
            ctx.write(n, T(getattr(s, n)))
        ctx.advance(g, 5)
        for n, v in zip(adn, adj):
            ctx.write(n, T(v))
        dJ = torch.zeros(wl.nx * wl.ny, dtype=torch.float64, device=DEV)
        ctx.adjoint_advance(0.5, 4, dJ)
        torch.cuda.synchronize()
        out.append([ctx.read(n).cpu().numpy() for n in fwd + adn] + [dJ.cpu().numpy()])
    for o in out[1:]:
        for a, b in zip(out[0], o):
            assert np.array_equal(a, b)


def _steady_run(wl, ty, spl, nf, na, prec="fp32"):
    ctx = lks.LKS(wl, precision=prec, device=DEV)
    ctx.set_tile_rows(ty)
    ctx.set_steps_per_launch(spl)
    assert ctx.launch_shape() == (ty, spl, spl)
    g = T(wl.gamma)
    d = torch.empty_like(g)
    ctx.forward(g, nf)
    J = ctx.objective()
    fields = [ctx.read(n).cpu().numpy() for n in ("drho", "ux", "uy")]
    ctx.backward(0.7, d, na)
    torch.cuda.synchronize()
    adj = [ctx.read(n).cpu().numpy() for n in ("adj_rho", "adj_vx", "adj_vy")]
    return J, fields, adj, d.cpu().numpy()


@pytest.mark.parametrize("ty", [4, 8])
@pytest.mark.parametrize("case", ["channel_70x37", "channel_65x9", "periodic_67x13"])
def test_two_steps_per_launch_give_the_same_bits(case, ty):
    """Two fused time steps per launch (tile + 4-node halo in LDS) against one
    step per launch: odd and even step counts, partial and merged tiles,
    corners, periodic wrap."""
    say(f"[gpu] two steps per launch {case} ty={ty}")
    wl = CASES[case]()
    for nf, na in ((7, 9), (12, 10)):
        ref = _steady_run(wl, ty, 1, nf, na)
        got = _steady_run(wl, ty, 2, nf, na)
        assert ref[0] == got[0]
        for a, b in zip(ref[1] + ref[2] + [ref[3]], got[1] + got[2] + [got[3]]):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("ty", [4, 8])
@pytest.mark.parametrize("case", ["channel_70x37", "periodic_67x13"])
def test_fp64_two_step_forward_gives_the_same_bits(case, ty):
    """The FP64 non-thermal forward with two steps per launch against one
    step per launch, odd and even step counts (the adjoint one step per
    launch in both)."""
    say(f"[gpu] FP64 two-step forward {case} ty={ty}")
    wl = CASES[case]()
    for nf in (7, 12):
        out = []
        for spl in (1, 2):
            ctx = lks.LKS(wl, precision="fp64", device=DEV)
            ctx.set_tile_rows(ty)
            ctx.set_steps_per_launch(spl, 1)
            assert ctx.launch_shape() == (ty, spl, 1)
            g = T(wl.gamma)
            d = torch.empty_like(g)
            ctx.forward(g, nf)
            J = ctx.objective()
            fields = [ctx.read(n).cpu().numpy() for n in ("drho", "ux", "uy")]
            ctx.backward(0.7, d, 5)
            torch.cuda.synchronize()
            out.append((J, fields + [d.cpu().numpy()]))
        assert out[0][0] == out[1][0]
        for a, b in zip(out[0][1], out[1][1]):
            assert np.array_equal(a, b)


def _steady_exchanger(mode):
    """Steady heat exchanger (heat source on) on a 70 x 70 grid: ragged
    tiles, corners, flux and Dirichlet ends; paper or exact adjoint."""
    wl = W.heat_exchanger(n=70, Re=20.0, sigma=3.0, seed=5, n_fwd=9, n_adj=11)
    wl.adjoint_mode = mode
    return wl


def _heated_periodic_box(mode):
    """Periodic thermal box 70 x 26 (tiles that are not full in x and y,
    wrapped halos), heated by the source and stirred by the Boussinesq
    force; paper or exact adjoint."""
    wl = W.periodic_box(70, 26, nu=0.08, thermal=True)
    wl.gamma = W.gamma_grf(70, 26, 3.0, 5)
    wl.alpha_max, wl.beta_max, wl.objective = 1.0, 0.1, W.OBJ_HEAT_EXCHANGE
    wl.gbeta, wl.T_ref = (0.0, 1e-4), 0.5
    wl.n_fwd, wl.n_adj, wl.adjoint_mode = 9, 11, mode
    return wl


@pytest.mark.parametrize("ty", [4, 8])
@pytest.mark.parametrize("mode", ["paper", "exact"])
@pytest.mark.parametrize("make", [_steady_exchanger, _heated_periodic_box])
def test_two_steps_per_launch_thermal_give_the_same_bits(make, mode, ty):
    """The thermal two-step kernels (new temperature of the first step kept
    beside the old one in LDS) against one step per launch, forward and
    adjoint, odd and even step counts."""
    wl = make(mode)
    say(f"[gpu] two steps per launch, thermal {wl.name} {mode} ty={ty}")
    out = []
    for spl in (1, 2):
        ctx = lks.LKS(wl, precision="fp32", device=DEV)
        ctx.set_tile_rows(ty)
        ctx.set_steps_per_launch(spl)
        assert ctx.launch_shape() == (ty, spl, spl)
        g = T(wl.gamma)
        d = torch.empty_like(g)
        ctx.forward(g, wl.n_fwd)
        J = ctx.objective()
        fields = [ctx.read(n).cpu().numpy() for n in ("drho", "ux", "uy", "T")]
        ctx.backward(0.7, d, wl.n_adj)
        torch.cuda.synchronize()
        adj = [ctx.read(n).cpu().numpy() for n in ("adj_rho", "adj_vx", "adj_vy", "adj_theta")]
        out.append((J, fields + adj + [d.cpu().numpy()]))
    assert out[0][0] == out[1][0]
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)


def test_two_steps_per_launch_full_size_512():
    """At full size the one-step kernel runs interior tiles through its
    branch-free variant, whose floating-point contraction may differ from the
    two-step kernel's, so the comparison is to FP32 rounding."""
    say("[gpu] two steps per launch 512x512, 300+301 steps")
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0)
    ref = _steady_run(wl, 8, 1, 300, 301)
    got = _steady_run(wl, 8, 2, 300, 301)
    assert abs(ref[0] - got[0]) <= 1e-6 * abs(ref[0])
    for a, b in zip(ref[1] + ref[2], got[1] + got[2]):
        assert rel(b, a) < 1e-5
    assert rel(got[3], ref[3]) < 1e-4


def test_autotune_picks_a_supported_height_and_keeps_results():
    say("[gpu] autotune 512x512")
    wl = W.steady_channel_grf(512, 512, Re=100.0, sigma=8.0, seed=0, n_fwd=100, n_adj=100)
    ctx = lks.LKS(wl, precision="fp32", device=DEV)
    g = T(wl.gamma)
    ty = ctx.autotune(g, 50)
    assert ty in (4, 8, 16)
    shape = ctx.launch_shape()
    assert shape[0] == ty and shape[1] in (1, 2) and shape[2] in (1, 2)
    d = torch.empty_like(g)
    ctx.forward(g, wl.n_fwd)
    J = ctx.objective()
    ctx.backward(1.0, d, wl.n_adj)
    ref = lks.LKS(wl, precision="fp32", device=DEV)
    ref.set_tile_rows(shape[0])
    ref.set_steps_per_launch(shape[1], shape[2])
    d2 = torch.empty_like(g)
    ref.forward(g, wl.n_fwd)
    J2 = ref.objective()
    ref.backward(1.0, d2, wl.n_adj)
    torch.cuda.synchronize()
    assert J == J2 and torch.equal(d, d2)
