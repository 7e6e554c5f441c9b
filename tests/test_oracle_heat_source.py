"""The heat source Q = beta_gamma (1 - T) (eq:heatsource, eq:betagamma) and
the heat-exchange objective J = -sum beta_gamma (1 - T)
(eq:objective_heatexchanger) in the oracle.

Readings pinned here: the source acts at the new level, so the zeroth moment
of eq:lbeg_ex gives T (1 + beta) = T* + beta; the adjoint term
dx dQ/dg_i T~ of eq:albeg_ex is implicit in T~ the same way
(T~ (1 + beta) = ...); the sensitivity adds dJ_O/dgamma - dx dQ/dgamma T~
(Sec. 2.5). In exact mode the division by 1 + beta moves to the propagated
Theta, and the unsteady gradient equals central differences of J."""
import numpy as np
import pytest

import oracle as O
from oracle import Problem, State, adjoint_equilibrium, adjoint_unsteady, alks_step
from oracle import forward, lks_step
from paper_2411_03090_amd import workloads as W


def test_source_coefficient_special_cases():
    """beta = bbar in the solid (gamma = 0), 0 in the fluid (gamma = 1), and
    beta' is the derivative of beta (central differences of the oracle's own
    beta at interior nodes; ring nodes are non-design)."""
    wl = W.heat_exchanger(n=12, Re=10.0, n_fwd=1, n_adj=1)
    wl.beta_max, wl.q_beta = 0.3, 0.2
    pb = Problem(wl)
    g = np.linspace(0.0, 1.0, 144).reshape(12, 12)
    b, db = O.source_coefficients(pb, g)
    b, db = b.reshape(12, 12), db.reshape(12, 12)
    inner = (slice(1, -1), slice(1, -1))
    assert b[0, :].max() == 0.0 and b[:, -1].max() == 0.0 and np.abs(db[0, :]).max() == 0.0
    g0 = np.zeros((12, 12))
    assert np.allclose(O.source_coefficients(pb, g0)[0].reshape(12, 12)[inner], 0.3, atol=1e-15)
    assert np.allclose(O.source_coefficients(pb, g0 + 1.0)[0], 0.0, atol=1e-16)
    e = 1e-6
    bp = O.source_coefficients(pb, g + e)[0].reshape(12, 12)
    bm = O.source_coefficients(pb, g - e)[0].reshape(12, 12)
    assert np.allclose(db[inner], ((bp - bm) / (2 * e))[inner], rtol=1e-7, atol=1e-9)
    assert np.all(db[inner] < 0.0)


@pytest.mark.parametrize("beta,T0", [(0.2, 0.0), (0.05, 0.7), (0.5, -0.3)])
def test_uniform_box_follows_the_implicit_source_update(beta, T0):
    """At rest with uniform T and beta the pull returns T, so
    T_{n+1} = (T_n + beta) / (1 + beta): T_n = 1 - (1 - T_0)(1 + beta)^-n,
    and the objective of a level is -N beta (1 - T_n)."""
    nx, ny = 8, 6
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.beta_max, wl.q_beta = 1.0, 0.1
    wl.objective = W.OBJ_HEAT_EXCHANGE
    pb = Problem(wl)
    N = nx * ny
    alpha, B, b = np.full(N, 0.4), np.full(N, 0.45), np.full(N, beta)
    s = State(np.zeros(N), np.zeros(N), np.zeros(N), np.full(N, T0))
    for n in range(1, 15):
        s = lks_step(pb, alpha, B, 1.0, s, b)
        want = 1.0 - (1.0 - T0) * (1.0 + beta) ** (-n)
        assert np.allclose(s.T, want, rtol=0, atol=2e-15)
        assert np.allclose(s.ux, 0.0, atol=0) and np.allclose(s.drho, 0.0, atol=0)
        J = O.level_objective(pb, s, b)
        assert J == pytest.approx(-N * beta * (1.0 - T0) * (1.0 + beta) ** (-n), rel=1e-13)


def test_source_acts_with_the_new_temperature():
    """Q is taken at t + dt: the step with the source differs from the one
    without by beta (1 - T*) / (1 + beta), T* the sourceless result, and not
    by beta (1 - T^n)."""
    nx, ny = 8, 6
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(0)
    s = State(np.zeros(N), 0.05 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.5 + 0.3 * rng.standard_normal(N))
    a, B, b = 0.5 * rng.random(N), np.full(N, 0.45), 0.3 * rng.random(N)
    s1 = lks_step(pb, a, B, 1.0, s, b)
    s0 = lks_step(pb, a, B, 1.0, s)
    assert np.allclose(s1.T - s0.T, b * (1.0 - s0.T) / (1.0 + b), rtol=0, atol=1e-15)
    assert np.max(np.abs(s1.T - s0.T - b * (1.0 - s.T))) > 1e-3
    assert np.array_equal(s1.ux, s0.ux) and np.array_equal(s1.drho, s0.drho)


def _dot_mismatch(mode, gb):
    """<L delta, (rho~, V, Theta)^{n+1}> against <delta, (rho~, V, Theta)^n>
    with L the (linear-by-symmetry) tangent of one LKS step."""
    nx, ny = 12, 10
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, gb, 0.3
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(4)
    a = 2.0 * rng.random(N)
    b = 0.8 * rng.random(N)
    B = np.full(N, 0.45)
    S = State(1e-2 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.05 * rng.standard_normal(N), rng.standard_normal(N))
    d = State(*(rng.standard_normal(N) for _ in range(4)))
    sh = lambda sg: State(S.drho + sg * d.drho, S.ux + sg * d.ux, S.uy + sg * d.uy,
                          S.T + sg * d.T)
    # the source term beta / (1 + beta) is constant and cancels in the difference
    Fp = lks_step(pb, a, B, 1.0, sh(1.0), b)
    Fm = lks_step(pb, a, B, 1.0, sh(-1.0), b)
    Ld = [(x - y) / 2 for x, y in ((Fp.drho, Fm.drho), (Fp.ux, Fm.ux), (Fp.uy, Fm.uy),
                                   (Fp.T, Fm.T))]
    S1 = lks_step(pb, a, B, 1.0, S, b)
    adj1 = [rng.standard_normal(N) for _ in range(9)]
    Vx, Vy, Th = adjoint_equilibrium(pb, B, S1.ux, S1.uy, adj1)
    lhs = adj1[0] @ Ld[0] + Vx @ Ld[1] + Vy @ Ld[2] + Th @ Ld[3]
    adj0 = alks_step(pb, a, B, S1, S, adj1, 0.0, 0.0, b, 0.0)
    Vx0, Vy0, Th0 = adjoint_equilibrium(pb, B, S.ux, S.uy, adj0)
    rhs = adj0[0] @ d.drho + Vx0 @ d.ux + Vy0 @ d.uy + Th0 @ d.T
    return abs(lhs - rhs) / abs(lhs)


@pytest.mark.parametrize("gb", [(0.0, 0.0), (0.004, -0.007)])
def test_exact_mode_is_the_transpose_with_the_source(gb):
    assert _dot_mismatch("exact", gb) < 1e-12


def test_paper_mode_is_not_the_transpose_with_the_source():
    """The paper divides T~ where it is formed, which is not the transpose of
    the division of T* (as for the Brinkman term)."""
    assert _dot_mismatch("paper", (0.0, 0.0)) > 1e-3


def _case(mode, obj, gb):
    nx, ny = 14, 12
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True, Pr=6)
    wl.mode, wl.objective = W.MODE_UNSTEADY, obj
    wl.Ks_over_Kf, wl.alpha_max = 1.0, 0.5
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, gb, 0.5
    wl.beta_max, wl.q_beta = 0.2, 0.1
    wl.mask = wl.mask.copy()
    wl.mask[3:8, 5] |= W.TAG_PROBE
    wl.gamma = np.clip(W.gamma_grf(nx, ny, 3.0, 4), 0.2, 1.0)
    n = 40
    wl.n_fwd, wl.ufac = n, np.ones(n + 1)
    j = np.arange(ny)[:, None] * np.ones((1, nx))
    i = np.arange(nx)[None, :] * np.ones((ny, 1))
    s0 = State(np.zeros(nx * ny), (0.02 * np.sin(2 * np.pi * j / ny)).ravel(),
               np.zeros(nx * ny), np.sin(2 * np.pi * i / nx).ravel())
    return wl, s0


def _adjoint_and_fd(mode, obj, gb, nodes=None):
    wl, s0 = _case(mode, obj, gb)
    pb = Problem(wl)
    n = wl.n_fwd
    _, _, traj = forward(pb, wl.gamma, n, store=True, state0=s0)
    _, sens = adjoint_unsteady(pb, wl.gamma, traj, 1.0)
    nodes = range(wl.nx * wl.ny) if nodes is None else nodes
    fd = []
    for k in nodes:
        vals = []
        for e in (1e-4, -1e-4):
            g = wl.gamma.copy().ravel()
            g[k] += e
            vals.append(forward(pb, g.reshape(wl.ny, wl.nx), n, state0=s0)[1])
        fd.append((vals[0] - vals[1]) / 2e-4)
    return sens[list(nodes)], np.array(fd)


@pytest.mark.parametrize("obj,gb", [(W.OBJ_HEAT_EXCHANGE, (0.0, 0.0)),
                                    (W.OBJ_HEAT_EXCHANGE, (0.0, 0.02)),
                                    (W.OBJ_HEAT, (0.0, 0.02))])
def test_exact_mode_gradient_with_the_source_equals_central_differences(obj, gb):
    """Exact to the truncation error of the differences (eps = 1e-4): this pins
    the source's forward reading, the heat-exchange objective and its seed,
    the explicit dJ_O/dgamma term and the -dQ/dgamma T~ term."""
    adj, fd = _adjoint_and_fd("exact", obj, gb, nodes=[78, 47, 116, 85, 152])
    assert np.max(np.abs(adj / fd - 1.0)) < 1e-6


def test_paper_mode_gradient_with_the_source_is_approximate():
    """The paper's implicit T~ is a continuous-adjoint approximation: over all
    nodes its gradient stays within 5 % (relative L2) of central
    differences here."""
    adj, fd = _adjoint_and_fd("paper", W.OBJ_HEAT_EXCHANGE, (0.0, 0.0))
    assert np.corrcoef(adj, fd)[0, 1] > 0.99
    assert np.linalg.norm(adj - fd) / np.linalg.norm(fd) < 0.1
