"""The Boussinesq force G = g beta (T - T_ref) (eq:boussinesqforce) in the
oracle: the forward LKS step takes u (1 + alpha) = U* + G at the new level
(eq:lbef_ex), and the adjoint adds its coupling to T~ (eq:albeg_ex; paper
mode) or to the propagated Theta (exact mode).

Pins: a uniform box under a uniform force follows the closed form of the
implicit update; in exact mode the ALKS step stays the transpose of the LKS
tangent with the force on, and the unsteady gradient equals central
differences of J."""
import numpy as np
import pytest

from oracle import Problem, State, adjoint_equilibrium, adjoint_unsteady, alks_step
from oracle import coefficients, forward, lks_step
from paper_2411_03090_amd import workloads as W

GB = (0.004, -0.007)


@pytest.mark.parametrize("a0", [0.0, 0.3])
def test_uniform_box_follows_the_implicit_force_update(a0):
    """Uniform state: U* = u and T stays, so u_{n+1} = (u_n + G) / (1 + alpha):
    u_n = u_inf + (u_0 - u_inf)(1 + alpha)^-n with u_inf = G / alpha, or
    u_0 + n G without Brinkman."""
    nx, ny = 8, 6
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.gbeta, wl.T_ref = GB, 0.25
    pb = Problem(wl)
    N = nx * ny
    alpha, B = np.full(N, a0), np.full(N, 0.45)
    T0 = 0.8
    u0 = np.array([0.01, -0.02])
    s = State(np.zeros(N), np.full(N, u0[0]), np.full(N, u0[1]), np.full(N, T0))
    G = np.array(GB) * (T0 - 0.25)
    for n in range(1, 13):
        s = lks_step(pb, alpha, B, 1.0, s)
        if a0 == 0.0:
            want = u0 + n * G
        else:
            uinf = G / a0
            want = uinf + (u0 - uinf) * (1.0 + a0) ** (-n)
        assert np.allclose(s.ux, want[0], rtol=0, atol=1e-15)
        assert np.allclose(s.uy, want[1], rtol=0, atol=1e-15)
        assert np.allclose(s.T, T0, rtol=0, atol=1e-15)
        assert np.allclose(s.drho, 0.0, rtol=0, atol=1e-15)


def test_force_acts_with_the_new_temperature():
    """eq:lbef_ex evaluates G at t + dt: the forced and unforced steps differ
    by g beta (T^{n+1} - T_ref) / (1 + alpha), not by the same with T^n."""
    nx, ny = 8, 6
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.gbeta, wl.T_ref = GB, 0.8
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(0)
    s = State(np.zeros(N), 0.05 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.8 + 0.3 * rng.standard_normal(N))
    a, B = 0.5 * rng.random(N), np.full(N, 0.45)
    s1 = lks_step(pb, a, B, 1.0, s)
    s0 = lks_step(Problem(W.periodic_box(nx, ny, nu=0.1, thermal=True)), a, B, 1.0, s)
    dT = s1.T - 0.8
    assert np.allclose(s1.ux - s0.ux, GB[0] * dT / (1 + a), rtol=0, atol=1e-16)
    assert np.allclose(s1.uy - s0.uy, GB[1] * dT / (1 + a), rtol=0, atol=1e-16)
    assert np.max(np.abs(s1.ux - s0.ux - GB[0] * (s.T - 0.8) / (1 + a))) > 1e-5


def _dot_mismatch(mode):
    nx, ny = 12, 10
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True)
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, GB, 0.3
    pb = Problem(wl)
    N = nx * ny
    rng = np.random.default_rng(4)
    a = 2.0 * rng.random(N)
    B = np.full(N, 0.45)
    S = State(1e-2 * rng.standard_normal(N), 0.05 * rng.standard_normal(N),
              0.05 * rng.standard_normal(N), rng.standard_normal(N))
    d = State(*(rng.standard_normal(N) for _ in range(4)))
    sh = lambda sg: State(S.drho + sg * d.drho, S.ux + sg * d.ux, S.uy + sg * d.uy,
                          S.T + sg * d.T)
    Fp = lks_step(pb, a, B, 1.0, sh(1.0))
    Fm = lks_step(pb, a, B, 1.0, sh(-1.0))
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


def test_exact_mode_is_the_transpose_with_the_force():
    assert _dot_mismatch("exact") < 1e-12


def _case(mode):
    nx, ny = 14, 12
    wl = W.periodic_box(nx, ny, nu=0.1, thermal=True, Pr=6)
    wl.mode, wl.objective = W.MODE_UNSTEADY, W.OBJ_HEAT
    wl.Ks_over_Kf, wl.alpha_max = 1.0, 0.5
    wl.adjoint_mode, wl.gbeta, wl.T_ref = mode, (0.0, 0.02), 0.5
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


def _adjoint_and_fd(mode, nodes=None):
    wl, s0 = _case(mode)
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


def test_exact_mode_gradient_with_the_force_equals_central_differences():
    adj, fd = _adjoint_and_fd("exact", nodes=[78, 47, 116, 85, 152])
    assert np.max(np.abs(adj / fd - 1.0)) < 1e-6


def test_paper_mode_gradient_with_the_force_is_approximate():
    """The paper's coupling 3 g beta . u~ and its Brinkman placement form a
    continuous-adjoint approximation: over all nodes the gradient stays
    highly correlated with central differences, with an error of the same
    order as without the force (12 % relative L2 at g beta = 0, 20 % here)."""
    adj, fd = _adjoint_and_fd("paper")
    assert np.corrcoef(adj, fd)[0, 1] > 0.95
    assert np.linalg.norm(adj - fd) / np.linalg.norm(fd) < 0.3
