"""The exact-discrete-adjoint mode of the oracle (a variant beside the ALKS
of Sec. 2.5). The forward velocity is u = U* / (1 + alpha) (eq:lbef_ex with
the Brinkman term implicit); its transpose divides the propagated
coefficient V of eq:afeq by 1 + alpha at the node where the velocity was
formed, and the Brinkman part of the sensitivity becomes
alpha' u.V / (1 + alpha).

The mode also replaces the product rule -B div q~ - grad B . q~ of eq:ageq
by the transpose of the forward B c_i.grad_h T, -div_h (B q~), and pairs the
conductivity term of the sensitivity with the levels whose equilibria the
steps use (0..N-1) while the Brinkman term pairs with the levels the steps
produce (1..N).

Pins: on periodic grids the ALKS step is then the exact transpose of the LKS
tangent for any alpha and any B (the paper's form is not), the unsteady
gradient equals central differences of J to their truncation error with a
conductivity contrast too (the paper's gradient does not), and the thermal
adjoint stays bounded where the paper's grows without bound."""
import numpy as np
import pytest

from oracle import Problem, State, adjoint_equilibrium, adjoint_unsteady, alks_step
from oracle import forward, lks_step
from paper_2411_03090_amd import workloads as W


def _dot_mismatch(mode, thermal, vary_B=False):
    nx, ny = 12, 10
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=thermal)
    wl.adjoint_mode = mode
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(3)
    a = 2.0 * rng.random(N)  # alpha in [0, 2)
    B = 0.05 + 0.4 * rng.random(N) if vary_B else np.full(N, 0.45)
    S = State(1e-2 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.05 * rng.standard_normal(N), rng.standard_normal(N))
    d = State(*(rng.standard_normal(N) for _ in range(4)))

    def shifted(sg):
        return State(S.drho + sg * d.drho, S.ux + sg * d.ux, S.uy + sg * d.uy, S.T + sg * d.T)

    # the step is quadratic in the state: L d = (F(S + d) - F(S - d)) / 2
    Fp = lks_step(pb, a, B, 1.0, shifted(1.0))
    Fm = lks_step(pb, a, B, 1.0, shifted(-1.0))
    Ld = [(x - y) / 2 for x, y in ((Fp.drho, Fm.drho), (Fp.ux, Fm.ux), (Fp.uy, Fm.uy),
                                   (Fp.T, Fm.T))]
    S1 = lks_step(pb, a, B, 1.0, S)
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    # the undivided V pairs with u in both modes' identity
    Vx, Vy, Th = adjoint_equilibrium(pb, B, S1.ux, S1.uy, adj1)
    lhs = adj1[0] @ Ld[0] + Vx @ Ld[1] + Vy @ Ld[2] + (Th @ Ld[3] if thermal else 0.0)
    adj0 = alks_step(pb, a, B, S1, S, adj1, 0.0, 0.0)
    Vx0, Vy0, Th0 = adjoint_equilibrium(pb, B, S.ux, S.uy, adj0)
    rhs = adj0[0] @ d.drho + Vx0 @ d.ux + Vy0 @ d.uy + (Th0 @ d.T if thermal else 0.0)
    return abs(lhs - rhs) / abs(lhs)


@pytest.mark.parametrize("thermal", [False, True])
def test_exact_mode_is_the_transpose_for_any_alpha(thermal):
    assert _dot_mismatch("exact", thermal) < 1e-12


def test_exact_mode_is_the_transpose_for_any_conductivity():
    assert _dot_mismatch("exact", True, vary_B=True) < 1e-12


@pytest.mark.parametrize("thermal", [False, True])
def test_paper_mode_is_not_the_transpose_with_brinkman(thermal):
    assert _dot_mismatch("paper", thermal) > 1e-4


def test_paper_mode_product_rule_is_not_the_transpose_for_varying_conductivity():
    """With alpha = 0 the paper's form differs from the transpose only through
    the product rule of eq:ageq."""
    assert _dot_mismatch_B_only("paper") > 1e-3
    assert _dot_mismatch_B_only("exact") < 1e-12


def _dot_mismatch_B_only(mode):
    nx, ny = 12, 10
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.adjoint_mode = mode
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(8)
    a = np.zeros(N)
    B = 0.05 + 0.4 * rng.random(N)
    S = State(1e-2 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.05 * rng.standard_normal(N), rng.standard_normal(N))
    d = State(*(rng.standard_normal(N) for _ in range(4)))
    sh = lambda sg: State(S.drho + sg * d.drho, S.ux + sg * d.ux, S.uy + sg * d.uy,
                          S.T + sg * d.T)
    Fp, Fm = lks_step(pb, a, B, 1.0, sh(1.0)), lks_step(pb, a, B, 1.0, sh(-1.0))
    Ld = [(x - y) / 2 for x, y in ((Fp.drho, Fm.drho), (Fp.ux, Fm.ux), (Fp.uy, Fm.uy),
                                   (Fp.T, Fm.T))]
    S1 = lks_step(pb, a, B, 1.0, S)
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx, Vy, Th = adjoint_equilibrium(pb, B, S1.ux, S1.uy, adj1)
    lhs = adj1[0] @ Ld[0] + Vx @ Ld[1] + Vy @ Ld[2] + Th @ Ld[3]
    adj0 = alks_step(pb, a, B, S1, S, adj1, 0.0, 0.0)
    Vx0, Vy0, Th0 = adjoint_equilibrium(pb, B, S.ux, S.uy, adj0)
    rhs = adj0[0] @ d.drho + Vx0 @ d.ux + Vy0 @ d.uy + Th0 @ d.T
    return abs(lhs - rhs) / abs(lhs)


def _periodic_unsteady(mode, ks=1.0):
    nx, ny = 14, 12
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True, Pr=6)
    wl.mode, wl.objective = W.MODE_UNSTEADY, W.OBJ_HEAT
    wl.Ks_over_Kf, wl.alpha_max = ks, 0.5  # alpha and (for ks != 1) B vary with gamma
    wl.adjoint_mode = mode
    wl.mask = wl.mask.copy()
    wl.mask[3:8, 5] |= W.TAG_PROBE
    wl.gamma = np.clip(W.gamma_grf(nx, ny, 3.0, 4), 0.2, 1.0)
    n = 40
    wl.n_fwd, wl.ufac = n, np.ones(n + 1)
    j = np.arange(ny)[:, None] * np.ones((1, nx))
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    s0 = State(np.zeros(nx * ny), (0.05 * np.sin(2 * np.pi * j / ny)).ravel(),
               (0.03 * np.cos(2 * np.pi * i / nx)).ravel(), np.sin(2 * np.pi * i / nx).ravel())
    return wl, s0


def _grad_vs_fd(mode, ks=1.0):
    wl, s0 = _periodic_unsteady(mode, ks)
    pb = Problem(wl)
    n = wl.n_fwd
    _, _, traj = forward(pb, wl.gamma, n, store=True, state0=s0)
    _, sens = adjoint_unsteady(pb, wl.gamma, traj, 1.0)
    sens = sens.reshape(wl.ny, wl.nx)
    pts = [(5, 8), (3, 5), (8, 4), (6, 1), (1, 7), (10, 12)]
    err = []
    for (jj, ii) in pts:
        vals = []
        for e in (1e-4, -1e-4):
            g = wl.gamma.copy()
            g[jj, ii] += e
            vals.append(forward(pb, g, n, state0=s0)[1])
        fd = (vals[0] - vals[1]) / 2e-4
        err.append(abs(sens[jj, ii] / fd - 1.0))
    return max(err)


@pytest.mark.parametrize("ks", [1.0, 3.0, 10.0])
def test_exact_mode_gradient_equals_central_differences(ks):
    # central differences with eps = 1e-4 carry an O(eps^2) truncation error;
    # ks = 10 puts B_s = 0 next to B_f = 0.45
    assert _grad_vs_fd("exact", ks) < 1e-6


@pytest.mark.parametrize("ks", [1.0, 10.0])
def test_paper_mode_gradient_is_approximate(ks):
    assert _grad_vs_fd("paper", ks) > 1e-4


# ---------------------------------------------------------------------------
# D3Q19
# ---------------------------------------------------------------------------
def _dot_mismatch_3d(mode, thermal, vary_B=False):
    from oracle import d3 as O3
    nx, ny, nz = 6, 5, 4
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=thermal)
    wl.adjoint_mode = mode
    pb = O3.Problem3(wl)
    N = nx * ny * nz
    rng = np.random.default_rng(5)
    a = 2.0 * rng.random(N)
    B = 0.05 + 0.4 * rng.random(N) if vary_B else np.full(N, 0.45)
    S = O3.State3(1e-2 * rng.standard_normal(N), 0.05 * rng.standard_normal(3 * N),
                  rng.standard_normal(N))
    d = O3.State3(rng.standard_normal(N), rng.standard_normal(3 * N), rng.standard_normal(N))
    sh = lambda sg: O3.State3(S.drho + sg * d.drho, S.u + sg * d.u, S.T + sg * d.T)
    Fp = O3.lks_step(pb, a, B, 1.0, sh(1.0))
    Fm = O3.lks_step(pb, a, B, 1.0, sh(-1.0))
    Ld = O3.State3((Fp.drho - Fm.drho) / 2, (Fp.u - Fm.u) / 2, (Fp.T - Fm.T) / 2)
    S1 = O3.lks_step(pb, a, B, 1.0, S)
    adj1 = [rng.standard_normal(N) for _ in range(14)]
    V1, Th1 = O3.adjoint_equilibrium(pb, B, S1.u, adj1)
    lhs = adj1[0] @ Ld.drho + V1 @ Ld.u + (Th1 @ Ld.T if thermal else 0.0)
    adj0 = O3.alks_step(pb, a, B, S1, S, adj1, 0.0, 0.0)
    V0, Th0 = O3.adjoint_equilibrium(pb, B, S.u, adj0)
    rhs = adj0[0] @ d.drho + V0 @ d.u + (Th0 @ d.T if thermal else 0.0)
    return abs(lhs - rhs) / abs(lhs)


@pytest.mark.parametrize("thermal", [False, True])
def test_exact_mode_is_the_transpose_for_any_alpha_3d(thermal):
    assert _dot_mismatch_3d("exact", thermal) < 1e-12


def test_exact_mode_is_the_transpose_for_any_conductivity_3d():
    assert _dot_mismatch_3d("exact", True, vary_B=True) < 1e-12
    assert _dot_mismatch_3d("paper", True, vary_B=True) > 1e-4


def test_paper_mode_is_not_the_transpose_with_brinkman_3d():
    assert _dot_mismatch_3d("paper", True) > 1e-4


@pytest.mark.parametrize("ks", [1.0, 4.0])
def test_exact_mode_gradient_equals_central_differences_3d(ks):
    from oracle import d3 as O3
    nx, ny, nz = 6, 5, 4
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=True, Pr=6.0)
    wl.mode, wl.objective = W.MODE_UNSTEADY, W.OBJ_HEAT
    wl.alpha_max, wl.Ks_over_Kf = 0.5, ks
    wl.adjoint_mode = "exact"
    wl.gamma = np.clip(0.6 + 0.4 * W.gaussian_random_field((nz, ny, nx), 1.5, 2), 0.1, 1.0)
    wl.mask = wl.mask.copy()
    wl.mask[1:3, 2:4, 3] |= W.TAG_PROBE
    n = 20
    wl.n_fwd, wl.ufac = n, np.ones(n + 1)
    pb = O3.Problem3(wl)
    rng = np.random.default_rng(2)
    N = pb.N
    s0 = O3.State3(np.zeros(N), 0.03 * rng.standard_normal(3 * N), rng.random(N))
    _, _, traj = O3.forward(pb, wl.gamma, n, store=True, state0=s0)
    _, sens = O3.adjoint_unsteady(pb, wl.gamma, traj, 1.0)
    sens = sens.reshape(nz, ny, nx)
    err = []
    for p in [(1, 2, 3), (2, 3, 1), (3, 1, 4), (0, 4, 2)]:
        vals = []
        for e in (1e-4, -1e-4):
            g = wl.gamma.copy()
            g[p] += e
            vals.append(O3.forward(pb, g, n, state0=s0)[1])
        err.append(abs(sens[p] / ((vals[0] - vals[1]) / 2e-4) - 1.0))
    assert max(err) < 1e-6
