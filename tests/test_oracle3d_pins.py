"""Pins of the D3Q19 oracle against facts fixed by the scheme and by the
mathematics, independent of the oracle itself:

* projection: D3Q19 summed along z is D2Q9 with its weights, so a z-invariant
  three-dimensional run reproduces the two-dimensional oracle (forward with
  boundaries, and the interior adjoint with its sensitivity);
* closed-form discrete dispersion of shear waves along every axis pair and of
  a fully three-dimensional thermal mode;
* periodic conservation of mass, momentum and heat;
* the adjoint dot-product identity;
* the face fill: covariance under the symmetries of the lattice and exact
  reproduction of a constant field at velocity and zero-flux faces;
* mirror symmetry of the heated-block duct;
* the gradient against central differences (periodic box: within the
  continuous-adjoint approximation; duct: recorded, parity unpinned).
"""
import itertools
import math

import numpy as np
import pytest

import oracle as O
from oracle import d3 as O3
from paper_2411_03090_amd import workloads as W

C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
W3 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)


def _nu_for_A(A):
    return 1.0 / 6.0 - 2.0 * A / 9.0


def test_lattice_projects_onto_d2q9():
    w2 = {}
    for c, w in zip(C3, W3):
        w2[(c[0], c[1])] = w2.get((c[0], c[1]), 0.0) + w
    want = {(0, 0): 4 / 9, (1, 0): 1 / 9, (0, 1): 1 / 9, (-1, 0): 1 / 9, (0, -1): 1 / 9,
            (1, 1): 1 / 36, (-1, 1): 1 / 36, (-1, -1): 1 / 36, (1, -1): 1 / 36}
    assert set(w2) == set(want)
    for k in want:
        assert w2[k] == pytest.approx(want[k], abs=1e-16)


# ---------------------------------------------------------------------------
# z-invariance: the three-dimensional oracle reproduces the two-dimensional one
# ---------------------------------------------------------------------------
def _state3_from_2d(s, nz):
    rep = lambda a: np.tile(a, nz)
    return O3.State3(rep(s.drho), np.concatenate([rep(s.ux), rep(s.uy), np.zeros(s.ux.size * nz)]),
                     rep(s.T))


@pytest.mark.parametrize("thermal", [False, True])
def test_z_invariant_channel_reproduces_2d_forward(thermal):
    nx, ny, nz, n = 17, 9, 3, 40
    wl = W.unsteady_thermal_channel(nx, ny, Re=40.0, sigma=2.0, seed=3, n_steps=n, period=15.0)
    wl.thermal = thermal
    if not thermal:
        wl.mask = wl.mask & np.uint8(0xF3)
        wl.mask[1:-1, -2] |= W.TAG_PROBE
    w3 = W.extrude_z(wl, nz)
    s2, J2, _ = O.forward(O.Problem(wl), wl.gamma, n)
    s3, J3, _ = O3.forward(O3.Problem3(w3), w3.gamma, n)
    N = nx * ny
    for name, a2, a3 in (("drho", s2.drho, s3.drho), ("ux", s2.ux, s3.u[:N * nz]),
                         ("uy", s2.uy, s3.u[N * nz:2 * N * nz]), ("T", s2.T, s3.T)):
        for l in range(nz):
            np.testing.assert_allclose(a3[l * N:(l + 1) * N], a2, rtol=1e-12, atol=1e-14,
                                       err_msg=name)
    assert np.abs(s3.u[2 * N * nz:]).max() < 1e-16
    if thermal:
        assert J3 / nz == pytest.approx(J2, rel=1e-12)


def _periodic2(nx, ny):
    wl = W.periodic_box(nx, ny, nu=0.08, thermal=True, Pr=6)
    wl.mode, wl.objective = W.MODE_UNSTEADY, W.OBJ_HEAT
    wl.Ks_over_Kf, wl.alpha_max = 3.0, 0.7
    wl.gamma = np.clip(W.gamma_grf(nx, ny, 2.0, 5), 0.05, 1.0)
    wl.mask = wl.mask.copy()
    wl.mask[2:5, 3] |= W.TAG_PROBE
    return wl


def test_z_invariant_periodic_adjoint_reproduces_2d():
    """Interior adjoint (alpha and B varying, coupling, seeds, sensitivity):
    z-invariant periodic runs agree. 3D moments (rho, u, s, T, q) map onto
    the 2D ones; u~_z, s~_xz, s~_yz and q~_z vanish."""
    nx, ny, nz, n = 9, 7, 2, 12
    wl = _periodic2(nx, ny)
    wl.n_fwd, wl.ufac = n, np.ones(n + 1)
    rng = np.random.default_rng(4)
    N = nx * ny
    s0 = O.State(1e-3 * rng.standard_normal(N), 0.03 * rng.standard_normal(N),
                 0.03 * rng.standard_normal(N), rng.random(N))
    pb2 = O.Problem(wl)
    _, J2, tr2 = O.forward(pb2, wl.gamma, n, store=True, state0=s0)
    adj2, sens2 = O.adjoint_unsteady(pb2, wl.gamma, tr2, 1.0)
    w3 = W.extrude_z(wl, nz)
    pb3 = O3.Problem3(w3)
    _, J3, tr3 = O3.forward(pb3, w3.gamma, n, store=True, state0=_state3_from_2d(s0, nz))
    adj3, sens3 = O3.adjoint_unsteady(pb3, w3.gamma, tr3, 1.0)
    assert J3 / nz == pytest.approx(J2, rel=1e-12)
    # 2D: rho ux uy sxx sxy syy T qx qy; 3D: rho u(3) sxx sxy sxz syy syz szz T q(3)
    pairs = [(0, 0), (1, 1), (2, 2), (3, 4), (4, 5), (5, 7), (6, 10), (7, 11), (8, 12)]
    scale = max(np.abs(a).max() for a in adj2)
    for f2, f3 in pairs:
        for l in range(nz):
            np.testing.assert_allclose(adj3[f3][l * N:(l + 1) * N], adj2[f2], rtol=0,
                                       atol=1e-12 * scale)
    for f3 in (3, 6, 8, 13):
        assert np.abs(adj3[f3]).max() < 1e-14 * scale
    for l in range(nz):
        np.testing.assert_allclose(sens3[l * N:(l + 1) * N], sens2, rtol=0,
                                   atol=1e-12 * np.abs(sens2).max())


# ---------------------------------------------------------------------------
# discrete dispersion
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("flow_axis,wave_axis,m,A", [(0, 2, 1, 0.3), (2, 1, 2, 0.6),
                                                     (1, 0, 1, 0.0), (1, 2, 3, 0.3)])
def test_shear_wave_decay_along_every_axis(flow_axis, wave_axis, m, A):
    """u_a = U sin(k x_b) (a != b) in a periodic box: exact solution with
    per-step factor 2/3 + cos(k)/3 + (2A/9) sin^2 k (the same as D2Q9, since
    D3Q19 summed along the third axis is D2Q9)."""
    dims = [6, 8, 10]
    nx, ny, nz = dims
    wl = W.periodic_box3(nx, ny, nz, nu=_nu_for_A(A))
    pb = O3.Problem3(wl)
    a, _, B, _ = O3.coefficients(pb, wl.gamma)
    n_b = dims[wave_axis]
    k = 2 * math.pi * m / n_b
    coords = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    xb = coords[2 - wave_axis].ravel().astype(float)
    N = nx * ny * nz
    U = 0.06
    u = np.zeros(3 * N)
    u[flow_axis * N:(flow_axis + 1) * N] = U * np.sin(k * xb)
    s = O3.State3(np.zeros(N), u, np.zeros(N))
    G = 2 / 3 + math.cos(k) / 3 + (2 * A / 9) * math.sin(k) ** 2
    for n in range(1, 5):
        s = O3.lks_step(pb, a, B, 1.0, s)
        want = np.zeros(3 * N)
        want[flow_axis * N:(flow_axis + 1) * N] = U * G ** n * np.sin(k * xb)
        np.testing.assert_allclose(s.u, want, atol=1e-15)
        assert np.abs(s.drho).max() < 1e-16


@pytest.mark.parametrize("kv", [(1, 0, 0), (1, 1, 1), (2, -1, 1), (0, 1, -2)])
def test_thermal_mode_decay_3d(kv):
    """With uniform u and B, T = Re exp(i k.x) advances by
    G_T = sum_i w_i [1 + 3 c_i.u + i B c_i.s(k)] exp(-i k.c_i) over the 19
    directions, s(k) = (sin k_x, sin k_y, sin k_z)."""
    nx, ny, nz = 8, 6, 10
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=True, Pr=6.0)
    pb = O3.Problem3(wl)
    a, _, B, _ = O3.coefficients(pb, wl.gamma)
    Bf = B[0]
    u0 = np.array([0.04, -0.03, 0.02])
    k = 2 * math.pi * np.array(kv) / np.array([nx, ny, nz])
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    phase = (k[0] * xx + k[1] * yy + k[2] * zz).ravel()
    sk = np.sin(k)
    G = sum(W3[q] * (1 + 3 * C3[q] @ u0 + 1j * Bf * (C3[q] @ sk)) * np.exp(-1j * (k @ C3[q]))
            for q in range(19))
    N = nx * ny * nz
    s = O3.State3(np.zeros(N), np.repeat(u0, N), np.cos(phase))
    for n in range(1, 4):
        s = O3.lks_step(pb, a, B, 1.0, s)
        np.testing.assert_allclose(s.T, np.real(G ** n * np.exp(1j * phase)), atol=3e-15)
        np.testing.assert_allclose(s.u, np.repeat(u0, N), atol=1e-16)


def test_periodic_conservation_3d():
    nx, ny, nz = 7, 6, 5
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=True)
    pb = O3.Problem3(wl)
    a, _, B, _ = O3.coefficients(pb, wl.gamma)
    rng = np.random.default_rng(8)
    N = nx * ny * nz
    s = O3.State3(0.01 * rng.standard_normal(N), 0.03 * rng.standard_normal(3 * N), rng.random(N))
    m0 = [s.drho.sum()] + [s.u[c * N:(c + 1) * N].sum() for c in range(3)] + [s.T.sum()]
    for _ in range(30):
        s = O3.lks_step(pb, a, B, 1.0, s)
    m1 = [s.drho.sum()] + [s.u[c * N:(c + 1) * N].sum() for c in range(3)] + [s.T.sum()]
    for x0, x1 in zip(m0, m1):
        assert abs(x1 - x0) < 1e-14 * max(N, abs(x0))


@pytest.mark.parametrize("thermal", [False, True])
def test_adjoint_dot_product_identity_3d(thermal):
    """<(rho~, V, Theta)^{n+1}, L_n d> = <(rho~, V, Theta)^n, d> on a periodic
    grid with alpha = 0 and uniform B; the step is quadratic, so
    L_n d = (F(S+d) - F(S-d))/2 exactly."""
    nx, ny, nz = 6, 5, 4
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=thermal)
    pb = O3.Problem3(wl)
    N = nx * ny * nz
    rng = np.random.default_rng(1)
    a = np.zeros(N)
    B = np.full(N, 0.45)
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
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


# ---------------------------------------------------------------------------
# face fill
# ---------------------------------------------------------------------------
def _signed_perms():
    for p in itertools.permutations(range(3)):
        for s in itertools.product((1, -1), repeat=3):
            M = np.zeros((3, 3), int)
            for r in range(3):
                M[r, p[r]] = s[r]
            yield M


def _dir_map(M):
    """index map q -> q' with c_q' = M c_q"""
    lut = {tuple(c): q for q, c in enumerate(C3)}
    return np.array([lut[tuple(M @ c)] for c in C3])


def _fill_problem(A, thermal):
    wl = W.periodic_box3(4, 4, 4, nu=_nu_for_A(A), thermal=thermal, Pr=6.0)
    wl.periodic_axes = 0
    return O3.Problem3(wl)


@pytest.mark.parametrize("cls", [W.FLOW_VELOCITY, W.FLOW_PRESSURE,
                                 W.FLOW_VELOCITY | W.THERM_FLUX | W.TAG_J_INLET,
                                 W.FLOW_PRESSURE | W.THERM_DIRICHLET | W.TAG_J_OUTLET])
def test_face_fill_is_covariant_under_lattice_symmetries(cls):
    """Mapping the known values and the normal by any of the 48 signed axis
    permutations maps the filled values the same way."""
    thermal = bool(cls & 12)
    pb = _fill_problem(0.3, thermal)
    rng = np.random.default_rng(2)
    n0 = np.array([0, -1, 0])
    u0 = np.array([0.02, 0.01, -0.03])
    fk = rng.standard_normal(19)
    gk = rng.standard_normal(19)
    known = C3 @ n0 <= 0
    fk[~known] = 0.0
    gk[~known] = 0.0
    f0, g0, _ = O3.boundary_fill(pb, cls, n0, 0.4, 0.7, u0, 0.3, fk, gk)
    for M in _signed_perms():
        mp = _dir_map(M)
        fkm = np.zeros(19)
        gkm = np.zeros(19)
        fkm[mp] = fk
        gkm[mp] = gk
        f1, g1, _ = O3.boundary_fill(pb, cls, M @ n0, 0.4, 0.7, M @ u0, 0.3, fkm, gkm)
        np.testing.assert_allclose(f1[mp], f0, atol=1e-12)
        if thermal:
            np.testing.assert_allclose(g1[mp], g0, atol=1e-12)


@pytest.mark.parametrize("A", [0.0, 0.3, 0.6])
def test_face_fill_reproduces_constants(A):
    """A constant known adjoint population c makes every residual vanish with
    f~_unknown = c at a velocity face (mu~ = -c (1 - 2A/3) n, by the isotropy
    sum_j w_j c_j c_j = I/3, plus the kappa~ T n term that the zero-flux
    condition adds to the flow rows) and g~_unknown = c at a zero-flux face
    with u.n = 0 (kappa~ = -c); least squares then returns exactly c."""
    pb = _fill_problem(A, True)
    for n in ([1, 0, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]):
        n = np.array(n)
        known = C3 @ n <= 0
        fk = np.where(known, 0.37, 0.0)
        gk = np.where(known, -1.3, 0.0)
        u = np.array([0.03, 0.01, 0.02]) * (1 - np.abs(n))
        f, g, mult = O3.boundary_fill(pb, W.FLOW_VELOCITY | W.THERM_FLUX, n, 0.45, 0.8, u,
                                      0.0, fk, gk)
        np.testing.assert_allclose(f, 0.37, atol=1e-13)
        np.testing.assert_allclose(g, -1.3, atol=1e-13)
        assert mult[3] == pytest.approx(1.3, abs=1e-13)
        np.testing.assert_allclose(mult[:3], -(0.37 * (1 - 2 * A / 3) - 1.3 * 0.8) * n,
                                   atol=1e-13)


# ---------------------------------------------------------------------------
# duct
# ---------------------------------------------------------------------------
def _small_duct(n=60, Re=20.0, seed=0):
    wl = W.heated_block_duct(18, 10, 12, Re=Re, Pr=0.71, sigma=2.0, seed=seed, n_steps=n)
    return wl


def test_duct_mirror_symmetry():
    """A design mirror-symmetric in z (the block and inflow are) gives u_x, T
    and the sensitivity symmetric and u_z antisymmetric."""
    wl = _small_duct(n=40)
    g = wl.gamma
    g[:] = 0.5 * (g + g[::-1])
    J, sens, s, adj = O3.gradient(wl)
    shp = (wl.nz, wl.ny, wl.nx)
    N = wl.nx * wl.ny * wl.nz
    ux = s.u[:N].reshape(shp)
    uz = s.u[2 * N:].reshape(shp)
    T = s.T.reshape(shp)
    np.testing.assert_allclose(ux, ux[::-1], atol=1e-14)
    np.testing.assert_allclose(uz, -uz[::-1], atol=1e-14)
    np.testing.assert_allclose(T, T[::-1], atol=1e-13)
    np.testing.assert_allclose(sens, sens[::-1], atol=1e-11 * np.abs(sens).max())
    assert np.abs(sens[wl.mask.reshape(shp) & W.TAG_SOLID > 0]).max() == 0.0


def test_duct_flow_develops_and_heats():
    """Sanity of the heated-block duct: flux through every cross-section is
    positive, the block is held at T = 1, and the objective is positive."""
    wl = _small_duct(n=150)
    pb = O3.Problem3(wl)
    s, J, _ = O3.forward(pb, wl.gamma, wl.n_fwd)
    N = wl.nx * wl.ny * wl.nz
    ux = s.u[:N].reshape(wl.nz, wl.ny, wl.nx)
    flux = ux[1:-1, 1:-1, :].sum(axis=(0, 1))
    assert np.all(flux > 0)
    blk = (wl.mask & W.THERM_DIRICHLET).astype(bool) & (wl.Tbar > 0)
    assert np.all(s.T.reshape(wl.nz, wl.ny, wl.nx)[blk] == 1.0)
    assert J > 0
    assert np.all(np.isfinite(s.u))


def test_gradient_matches_fd_periodic_thermal_3d():
    """Fully three-dimensional periodic thermal sweep (alpha' and B' terms,
    coupling, seeds): ALKS agrees with central differences within the
    continuous-adjoint approximation (< 25 % per node here; the identity is
    exact only for alpha = 0 and uniform B, see the dot-product pin)."""
    nx, ny, nz = 8, 7, 6
    wl = W.periodic_box3(nx, ny, nz, nu=0.1, thermal=True, Pr=6)
    wl.mode, wl.objective = W.MODE_UNSTEADY, W.OBJ_HEAT
    wl.Ks_over_Kf, wl.alpha_max = 4.0, 0.05
    wl.mask = wl.mask.copy()
    wl.mask[1:4, 2:5, 3] |= W.TAG_PROBE
    wl.gamma = np.clip(0.6 + 0.4 * W.gaussian_random_field((nz, ny, nx), 1.5, 3), 0.2, 1.0)
    n = 40
    wl.n_fwd, wl.ufac = n, np.ones(n + 1)
    pb = O3.Problem3(wl)
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    N = nx * ny * nz
    u0 = np.concatenate([(0.05 * np.sin(2 * np.pi * yy / ny)).ravel(),
                         (0.03 * np.cos(2 * np.pi * zz / nz)).ravel(),
                         (0.02 * np.sin(2 * np.pi * xx / nx)).ravel()])
    s0 = O3.State3(np.zeros(N), u0, np.sin(2 * np.pi * xx / nx).ravel())
    _, _, traj = O3.forward(pb, wl.gamma, n, store=True, state0=s0)
    _, sens = O3.adjoint_unsteady(pb, wl.gamma, traj, 1.0)
    sens = sens.reshape(nz, ny, nx)
    pts = [(2, 3, 4), (1, 2, 3), (4, 5, 1), (0, 0, 6), (3, 1, 2)]
    adj, fd = [], []
    for p in pts:
        vals = []
        for e in (1e-5, -1e-5):
            g = wl.gamma.copy()
            g[p] += e
            vals.append(O3.forward(pb, g, n, state0=s0)[1])
        fd.append((vals[0] - vals[1]) / 2e-5)
        adj.append(sens[p])
    adj, fd = np.array(adj), np.array(fd)
    assert np.all(np.sign(adj) == np.sign(fd))
    assert np.all(np.abs(adj / fd - 1.0) < 0.25)


@pytest.mark.slow
def test_duct_gradient_vs_fd_is_recorded():
    """Duct with the least-squares face fill (parity unpinned): ALKS is
    correlated with central differences of the heat objective."""
    wl = _small_duct(n=60, Re=10.0, seed=1)
    J, sens, _, _ = O3.gradient(wl)
    rng = np.random.default_rng(1)
    inner = np.argwhere((W._ends3(wl.nx, wl.ny, wl.nz, 0) == 0) & ~(wl.mask & W.TAG_SOLID > 0))
    pts = [tuple(inner[i]) for i in rng.choice(len(inner), 8, replace=False)]
    adj, fd = [], []
    for p in pts:
        vals = []
        for e in (1e-5, -1e-5):
            g = wl.gamma.copy()
            g[p] += e
            vals.append(O3.objective(wl, g))
        fd.append((vals[0] - vals[1]) / 2e-5)
        adj.append(sens[p])
    adj, fd = np.array(adj), np.array(fd)
    corr = np.corrcoef(adj, fd)[0, 1]
    print("duct ALKS/FD:", adj / fd, "corr", corr)
    assert corr > 0.9
