"""Prescribed heat flux -q.n = qbar (Sec. 2.4) and the heat-sink objective
(eq:objective_heatsink) in the oracle.

Pins: from a uniform state at rest one step raises exactly the heated nodes
by qbar (the closure T (1 + u.n) = S0 + 2 S+ + qbar); the least-squares
zero-flux completion with a boundary seed s has, at B = 0, the closed form
"each unknown = mean of the three known populations moving inwards - 2 s";
the D3Q19 face closure is the same. The gradient of the heat-sink objective
against central differences is recorded (parity with the exact derivative
is unpinned at boundaries, as for the other boundary objectives)."""
import numpy as np
import pytest

import oracle as O
from oracle import d3 as O3
from paper_2411_03090_amd import workloads as W


def _adiabatic_cavity(n=14, q0=0.02):
    wl = W.heat_sink(n=n, n_steps=10, q0=q0, Ks_over_Kf=1.0)
    wl.gbeta = (0.0, 0.0)
    m = wl.mask.copy()
    sel = (m & 3) == W.FLOW_VELOCITY
    m[sel] = (m[sel] & 0xF3) | W.THERM_FLUX
    wl.mask = m
    return wl


@pytest.mark.parametrize("T0", [0.0, 0.4])
def test_one_step_from_rest_adds_the_flux_at_heated_nodes(T0):
    wl = _adiabatic_cavity()
    n = wl.nx
    pb = O.Problem(wl)
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    N = n * n
    s = O.State(np.zeros(N), np.zeros(N), np.zeros(N), np.full(N, T0))
    s1 = O.lks_step(pb, a, B, 1.0, s)
    heated = (wl.mask.ravel() & W.TAG_PROBE) != 0
    assert np.allclose(s1.T[heated], T0 + 0.02, rtol=0, atol=1e-15)
    assert np.allclose(s1.T[~heated], T0, rtol=0, atol=1e-15)
    assert s1.T.sum() - s.T.sum() == pytest.approx(0.02 * heated.sum(), rel=1e-12)
    assert np.array_equal(s1.ux, s.ux) and np.array_equal(s1.uy, s.uy)


def test_heat_sink_objective_is_the_mean_heated_temperature():
    wl = W.heat_sink(n=16, n_steps=10)
    pb = O.Problem(wl)
    rng = np.random.default_rng(2)
    N = 16 * 16
    s = O.State(np.zeros(N), np.zeros(N), np.zeros(N), rng.random(N))
    heated = (wl.mask.ravel() & W.TAG_PROBE) != 0
    assert O.level_objective(pb, s) == pytest.approx(s.T[heated].mean(), rel=1e-14)


@pytest.mark.parametrize("seed", [0.0, 0.3, -1.1])
def test_zero_flux_fill_with_a_seed_closed_form(seed):
    """Bottom wall (n = (0,-1)), u = 0, B = 0: the thermal rows are
    (n.c_i)(g~_i + kappa~) + s. The three rows along the wall leave s; the
    rows of the unknown directions 4, 7, 8 vanish with g~ = -kappa~ - s; the
    rows of the known directions 2, 5, 6 then give kappa~ = s - their mean,
    so every unknown equals the mean of g~_2, g~_5, g~_6 minus 2 s."""
    wl = _adiabatic_cavity()
    pb = O.Problem(wl)
    rng = np.random.default_rng(5)
    fk, gk = rng.standard_normal(9), rng.standard_normal(9)
    m = W.FLOW_VELOCITY | W.THERM_FLUX
    _, g, mult = O.boundary_fill(pb, m, (0, -1), 0.0, 0.7, (0.0, 0.0), 0.0, fk, gk, seed_T=seed)
    want = (gk[2] + gk[5] + gk[6]) / 3.0 - 2.0 * seed
    assert np.allclose(g[[4, 7, 8]], want, rtol=0, atol=1e-13)
    assert mult[2] == pytest.approx(seed - (gk[2] + gk[5] + gk[6]) / 3.0, abs=1e-13)
    # the known populations are left as they were
    assert np.array_equal(g[[0, 1, 2, 3, 5, 6]], gk[[0, 1, 2, 3, 5, 6]])


def test_d3q19_flux_face_matches_the_z_invariant_d2q9_step():
    """The D3Q19 face closure with qbar: a z-invariant run of the adiabatic
    cavity (periodic along z) equals the D2Q9 step, heated nodes included."""
    wl = _adiabatic_cavity(n=12)
    wl.Tbar = wl.Tbar.copy()
    wl3 = W.extrude_z(wl, 4)
    pb, pb3 = O.Problem(wl), O3.Problem3(wl3)
    rng = np.random.default_rng(3)
    N = 12 * 12
    s = O.State(1e-3 * rng.standard_normal(N), np.zeros(N), np.zeros(N), rng.random(N))
    a, _, B, _ = O.coefficients(pb, wl.gamma)
    s1 = O.lks_step(pb, a, B, 1.0, s)
    a3, _, B3, _ = O3.coefficients(pb3, wl3.gamma)
    rep = lambda v: np.tile(v, 4)
    u3 = np.concatenate([rep(s.ux), rep(s.uy), np.zeros(4 * N)])
    t1 = O3.lks_step(pb3, a3, B3, 1.0, O3.State3(rep(s.drho), u3, rep(s.T)))
    assert np.allclose(t1.T.reshape(4, N), s1.T[None, :], rtol=0, atol=1e-14)
    assert np.allclose(t1.drho.reshape(4, N), s1.drho[None, :], rtol=0, atol=1e-14)


def test_heat_sink_gradient_vs_fd_is_recorded():
    """Unsteady heat sink (18 x 18, 150 steps, uniform conductivity, Ra = 2e4),
    every design node within a few cells of the heated boundary: the ALKS
    gradient of the mean heated temperature correlates with central
    differences (0.96 measured) but not in magnitude (relative L2 0.9): next
    to the heated boundary the paper's boundary treatment is approximate
    (parity unpinned there; the check of Sec. 2.6 below pins the interior)."""
    n = 18
    wl = W.heat_sink(n=n, n_steps=150, Ra=2e4, Ks_over_Kf=1.0, sigma=3.0, seed=1)
    J, sens, _, _ = O.gradient(wl)
    ks = [j * n + i for j in range(1, n - 1, 2) for i in range(1, n - 1, 2)]
    fd = []
    for k in ks:
        v = []
        for e in (1e-4, -1e-4):
            g = wl.gamma.copy().ravel()
            g[k] += e
            v.append(O.objective(wl, g.reshape(n, n)))
        fd.append((v[0] - v[1]) / 2e-4)
    fd = np.array(fd)
    adj = sens.ravel()[ks]
    assert np.corrcoef(adj, fd)[0, 1] > 0.9


@pytest.mark.parametrize("Ks,band", [(1.0, 0.15), (10.0, 0.6)])
def test_gradient_matches_fd_on_the_papers_natural_convection_check(Ks, band):
    """The natural-convection check of Sec. 2.6 (140 x 80 cells, walls at
    T = 0 on three sides, a heated 4-cell patch on the adiabatic bottom, the
    80 x 50 design domain at gamma = 0.9 with its 40 x 25 core at 0.1), with
    the heat-sink objective and physics of Sec. 3.4 (Ra = 2e5, Pr = 6) over
    10000 steps. Along the design domain's centre line the ALKS gradient
    follows central differences (eq:sensfdm, eps = 1e-3), as the paper
    reports (fair agreement, errors at the gamma interface). Measured,
    uniform conductivity: correlation 0.97, median ratio 1.02, relative L2
    0.10 over 13 nodes; K_s = 10 K_f: correlation 0.97, ratios 0.7-1.1 off the
    core and 0.2 inside it (the conductivity term in the solid, an error of
    the continuous adjoint the paper notes at the interface). This fixes the
    boundary seed of the heat-sink objective (through the heated node's flux
    closure); the literal uniform row seed gives correlation 0.5 and median
    ratio 0.05 here."""
    wl = W.sensitivity_check_natural_convection(Ks_over_Kf=Ks, n_steps=10000)
    J, sens, _, _ = O.gradient(wl, checkpoint=101)
    jc, eps = 40, 1e-3
    pts = [38, 50, 92, 104] if Ks > 1 else [38, 62, 80, 98]
    fd = []
    for i in pts:
        v = []
        for e in (eps, -eps):
            g = wl.gamma.copy()
            g[jc, i] += e
            v.append(O.objective(wl, g))
        fd.append((v[0] - v[1]) / (2 * eps))
    fd = np.array(fd)
    adj = sens[jc, pts]
    assert np.all(np.sign(adj) == np.sign(fd))
    assert np.all(np.abs(adj / fd - 1.0) < band)
