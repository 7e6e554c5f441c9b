"""Pins of the oracle's adjoint boundary completions other than the printed
velocity-node form (which test_oracle_pins.py pins against eq:ftilde).

Each boundary condition of Appendix A is a set of Q equations, one per
direction i, that the least squares of Sec. 2.5 satisfies as well as it can:

  pressure node (eq:afboundaryp, with -kappa~ T (c_i.n) at p-and-q nodes,
  eq:afboundarypq):
      (n.c_i) f~_i - 2A sum_j w_j (n.c_j)(c_j.c_i) f~_j
      + lambda~ + mu~_s (c_i.t) - kappa~ T (c_i.n) + s_i
  prescribed temperature (eq:agboundaryT):
      (n.c_i) g~_i - B (n.q~) + eta~ + s_T
  prescribed heat flux (eq:agboundaryq):
      (n.c_i) g~_i - B (n.q~) + kappa~ (c_i - u).n + s_T

with q~ = sum_j w_j c_j g~_j (eq:agq) and the s~ of the printed conditions
expanded through eq:afs. The unknowns are the populations with c_i.n > 0 and
the multipliers. The tests write these rows out here, independently of the
oracle, and check the oracle's completions three ways:
  * closed forms where the rows admit one (derived in each docstring);
  * the optimality condition of least squares, K^T r = 0, where K holds the
    derivatives of the rows with respect to the unknowns and r the residual
    at the oracle's solution -- a dropped or mis-signed term in the oracle's
    rows leaves a residual that is not orthogonal to the test's columns;
  * the known populations pass through unchanged.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
import oracle.d3 as O3
from paper_2411_03090_amd import workloads as W

CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
C2 = np.stack([CX, CY], axis=1)
W2 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
C3 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
               [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
               [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
W3 = np.array([1 / 3] + [1 / 18] * 6 + [1 / 36] * 12)
NORMALS2 = [(-1, 0), (1, 0), (0, -1), (0, 1)]
NORMALS3 = [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def _nu_for_A(A):
    return 1.0 / 6.0 - 2.0 * A / 9.0


def _problem2(A=0.3, thermal=True):
    wl = W.steady_channel_uniform(8, 8, Re=10, seed=0, n_fwd=1, n_adj=1)
    wl.nu = _nu_for_A(A)
    wl.thermal = thermal
    return O.Problem(wl)


def _problem3(A=0.3, thermal=True):
    wl = W.periodic_box3(4, 4, 4, nu=_nu_for_A(A), thermal=thermal, Pr=6.0)
    wl.periodic_axes = 0
    return O3.Problem3(wl)


def _known_random(rng, cn, Q):
    v = rng.standard_normal(Q)
    v[cn > 0] = 0.0
    return v


# ---------------------------------------------------------------------------
# rows of the boundary conditions, written out from Appendix A
# ---------------------------------------------------------------------------
def _thermal_rows(C, Wt, n, B, u, kind, s_T):
    """Residual of the thermal condition as an affine map of the full g~
    vector and the multiplier: r = Mg g~ + m * col + s_T."""
    cn = C @ np.asarray(n)
    Q = len(cn)
    Mg = np.diag(cn.astype(float)) - B * np.outer(np.ones(Q), Wt * cn)
    if kind == "dirichlet":
        col = np.ones(Q)
    else:
        col = cn - float(np.dot(u, n))
    return cn, Mg, col


def _flow_rows(C, Wt, n, A, kind):
    """Flow condition: r = M f~ + (multiplier columns) x + const."""
    cn = C @ np.asarray(n)
    M = np.diag(cn.astype(float)) - 2.0 * A * (C @ C.T) * (Wt * cn)[None, :]
    if kind == "velocity":
        cols = C.astype(float)
    else:
        t = np.array([-n[1], n[0]])
        cols = np.stack([np.ones(len(cn)), C @ t], axis=1).astype(float)
    return cn, M, cols


# ---------------------------------------------------------------------------
# prescribed temperature
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n", NORMALS2)
def test_dirichlet_fill_closed_form_2d(n):
    """eq:agboundaryT. The terms -B (n.q~) + eta~ + s_T are the same in every
    row, so write them as one number E. The three rows along the wall
    (c.n = 0) read E; the unknown rows (c.n = 1) read g~_i + E and vanish with
    g~_i = -E; the rows of the known populations moving inwards (c.n = -1)
    read E - g~_k. Least squares over E then gives 6E = sum of those known
    g~_k: every unknown equals -(sum of g~ with c.n = -1)/6, whatever B and
    the seed are, and eta~ = E + B (n.q~) - s_T with q~ of the completed set."""
    pb = _problem2()
    rng = np.random.default_rng(17)
    cn = C2 @ np.array(n)
    for B in (0.0, 0.45, -0.3):
        for seed_T in (0.0, 0.8):
            fk = _known_random(rng, cn, 9)
            gk = _known_random(rng, cn, 9)
            u = rng.standard_normal(2) * 0.05
            m = W.FLOW_VELOCITY | W.THERM_DIRICHLET
            _, g, mult = O.boundary_fill(pb, m, n, B, 0.6, u, 0.0, fk, gk, seed_T=seed_T)
            E = gk[cn < 0].sum() / 6.0
            np.testing.assert_allclose(g[cn > 0], -E, rtol=0, atol=1e-13)
            assert np.array_equal(g[cn <= 0], gk[cn <= 0])
            qn = float(np.dot(W2 * cn, g))
            assert mult[2] == pytest.approx(E + B * qn - seed_T, abs=1e-13)


@pytest.mark.parametrize("n", NORMALS3)
def test_dirichlet_fill_closed_form_3d(n):
    """The same argument on a D3Q19 face: 9 rows with c.n = 0, 5 unknown rows
    and 5 known rows give 14E = sum of the five known g~ with c.n = -1, every
    unknown -E, and eta~ = E + B (n.q~)."""
    pb = _problem3()
    rng = np.random.default_rng(23)
    cn = C3 @ np.array(n)
    for B in (0.0, 0.0775, 0.45):
        fk = _known_random(rng, cn, 19)
        gk = _known_random(rng, cn, 19)
        u = rng.standard_normal(3) * 0.05
        m = W.FLOW_VELOCITY | W.THERM_DIRICHLET
        _, g, mult = O3.boundary_fill(pb, m, n, B, 0.6, u, 0.0, fk, gk)
        E = gk[cn < 0].sum() / 14.0
        np.testing.assert_allclose(g[cn > 0], -E, rtol=0, atol=1e-13)
        assert np.array_equal(g[cn <= 0], gk[cn <= 0])
        qn = float(np.dot(W3 * cn, g))
        assert mult[3] == pytest.approx(E + B * qn, abs=1e-13)


# ---------------------------------------------------------------------------
# prescribed heat flux, general B and u.n
# ---------------------------------------------------------------------------
def _thermal_optimality(C, Wt, n, B, u, seed_T, g, kappa):
    cn, Mg, col = _thermal_rows(C, Wt, n, B, u, "flux", seed_T)
    r = Mg @ g + kappa * col + seed_T
    K = np.concatenate([Mg[:, cn > 0], col[:, None]], axis=1)
    return K.T @ r, np.abs(K).max() * (np.abs(g).max() + abs(kappa) + abs(seed_T))


@pytest.mark.parametrize("n", NORMALS2)
def test_zero_flux_fill_is_the_least_squares_solution_2d(n):
    """eq:agboundaryq with B != 0 and u.n != 0 (the outlet of a channel):
    the oracle's completed g~ and kappa~ make the residual orthogonal to the
    derivatives of every row with respect to the unknowns. With the rows
    being of full column rank this is the unique generalized-inverse
    solution."""
    pb = _problem2()
    rng = np.random.default_rng(29)
    cn = C2 @ np.array(n)
    for B in (0.45, 0.2, -0.1):
        for seed_T in (0.0, -0.7):
            fk = _known_random(rng, cn, 9)
            gk = _known_random(rng, cn, 9)
            u = rng.standard_normal(2) * 0.08
            m = W.FLOW_PRESSURE | W.THERM_FLUX
            _, g, mult = O.boundary_fill(pb, m, n, B, 0.6, u, 0.0, fk, gk, seed_T=seed_T)
            assert np.array_equal(g[cn <= 0], gk[cn <= 0])
            KTr, scale = _thermal_optimality(C2, W2, n, B, u, seed_T, g, mult[2])
            assert np.abs(KTr).max() < 1e-13 * scale
            # a dropped B term (or a wrong sign of u.n) would not be optimal
            KTr_wrong, _ = _thermal_optimality(C2, W2, n, 0.0, -u, seed_T, g, mult[2])
            if B != 0.0:
                assert np.abs(KTr_wrong).max() > 1e-6


@pytest.mark.parametrize("n", NORMALS3)
def test_zero_flux_fill_is_the_least_squares_solution_3d(n):
    pb = _problem3()
    rng = np.random.default_rng(31)
    cn = C3 @ np.array(n)
    for B in (0.0775, 0.45):
        fk = _known_random(rng, cn, 19)
        gk = _known_random(rng, cn, 19)
        u = rng.standard_normal(3) * 0.08
        m = W.FLOW_PRESSURE | W.THERM_FLUX
        _, g, mult = O3.boundary_fill(pb, m, n, B, 0.6, u, 0.0, fk, gk)
        assert np.array_equal(g[cn <= 0], gk[cn <= 0])
        KTr, scale = _thermal_optimality(C3, W3, n, B, u, 0.0, g, mult[3])
        assert np.abs(KTr).max() < 1e-13 * scale


# ---------------------------------------------------------------------------
# pressure outlet
# ---------------------------------------------------------------------------
# The right-side pressure node (n = (1, 0), t = (0, 1)) at A = 3/10, solved in
# exact rational arithmetic from the nine rows of eq:afboundaryp: the unknowns
# f~1, f~5, f~8 and the multipliers lambda~, mu~_s as linear forms in the
# known f~3, f~6, f~7 (the populations moving inwards; f~0, f~2, f~4 drop out).
OUTLET_A03 = {
    "f1": (Fraction(-29, 879), Fraction(-98, 879), Fraction(-98, 879)),
    "f5": (Fraction(-50, 879), Fraction(-1373, 3516), Fraction(385, 3516)),
    "f8": (Fraction(-50, 879), Fraction(385, 3516), Fraction(-1373, 3516)),
    "lam": (Fraction(112, 879), Fraction(136, 879), Fraction(136, 879)),
    "mus": (Fraction(0), Fraction(9, 40), Fraction(-9, 40)),
}


def _exact_outlet_forms(A):
    """Exact least-squares solution of the right-side pressure rows at a
    rational A, by Gauss-Jordan elimination on the normal equations in
    Fractions: for each known direction k, the solution with f~_k = 1."""
    n = (1, 0)
    t = (0, 1)
    cn = [int(CX[q] * n[0] + CY[q] * n[1]) for q in range(9)]
    w = [Fraction(4, 9)] + [Fraction(1, 9)] * 4 + [Fraction(1, 36)] * 4
    unk = [q for q in range(9) if cn[q] > 0]

    def M(r, q):
        cc = int(CX[q] * CX[r] + CY[q] * CY[r])
        return (cn[r] if r == q else 0) - 2 * A * w[q] * cn[q] * cc

    cols = [[M(r, q) for r in range(9)] for q in unk]
    cols += [[Fraction(1)] * 9, [Fraction(int(CX[r] * t[0] + CY[r] * t[1])) for r in range(9)]]
    nc = len(cols)
    G = [[sum(cols[a][r] * cols[b][r] for r in range(9)) for b in range(nc)] for a in range(nc)]
    out = {}
    for k in (3, 6, 7):
        b = [M(r, k) for r in range(9)]
        m = [G[a][:] + [-sum(cols[a][r] * b[r] for r in range(9))] for a in range(nc)]
        for p in range(nc):
            piv = next(r for r in range(p, nc) if m[r][p] != 0)
            m[p], m[piv] = m[piv], m[p]
            for r in range(nc):
                if r != p and m[r][p] != 0:
                    f = m[r][p] / m[p][p]
                    m[r] = [x - f * y for x, y in zip(m[r], m[p])]
        out[k] = [m[i][nc] / m[i][i] for i in range(nc)]
    return out


def test_outlet_fill_closed_form_at_A_three_tenths():
    """The oracle's outlet fill at A = 3/10 equals the rational closed form
    above, which the exact elimination reproduces."""
    exact = _exact_outlet_forms(Fraction(3, 10))
    for a, name in enumerate(("f1", "f5", "f8", "lam", "mus")):
        assert tuple(exact[k][a] for k in (3, 6, 7)) == OUTLET_A03[name], name
    pb = _problem2(A=0.3, thermal=False)
    rng = np.random.default_rng(37)
    cn = C2 @ np.array([1, 0])
    for _ in range(5):
        f = _known_random(rng, cn, 9)
        fk, _, mult = O.boundary_fill(pb, W.FLOW_PRESSURE, (1, 0), 0.0, 0.0, (0.02, 0.0), 0.0,
                                      f, np.zeros(9))
        got = {"f1": fk[1], "f5": fk[5], "f8": fk[8], "lam": mult[0], "mus": mult[1]}
        for name, forms in OUTLET_A03.items():
            want = sum(float(c) * f[k] for c, k in zip(forms, (3, 6, 7)))
            assert got[name] == pytest.approx(want, abs=1e-13), name
        assert np.array_equal(fk[cn <= 0], f[cn <= 0])


@pytest.mark.parametrize("A", [0.0, 0.3, 0.7])
@pytest.mark.parametrize("kind", ["velocity", "pressure"])
def test_flow_fill_is_the_least_squares_solution(A, kind):
    """Velocity and pressure nodes, with and without the zero-flux coupling
    -kappa~ T (c_i.n) (eq:afboundaryuq, eq:afboundarypq) and a pressure-drop
    seed on every row: the oracle's completion and multipliers make the
    residual orthogonal to every column of the rows written out here."""
    pb = _problem2(A=A)
    rng = np.random.default_rng(41)
    for n in NORMALS2:
        cn, M, cols = _flow_rows(C2, W2, n, A, kind)
        for thermal_flux in (False, True):
            for seed in (0.0, 0.9):
                fk = _known_random(rng, cn, 9)
                gk = _known_random(rng, cn, 9)
                u = np.zeros(2) if kind == "velocity" else 0.03 * np.array(n)
                Tn, B = 0.7, 0.45
                m = (W.FLOW_VELOCITY if kind == "velocity" else W.FLOW_PRESSURE) | W.TAG_J_INLET
                if thermal_flux:
                    m |= W.THERM_FLUX
                f, g, mult = O.boundary_fill(pb, m, n, B, Tn, u, seed, fk, gk)
                kappa = mult[2] if thermal_flux else 0.0
                # the boundary seed per unit pressure on an inlet-tagged node
                s = seed
                r = M @ f + cols @ mult[:2] - kappa * Tn * cn + s
                K = np.concatenate([M[:, cn > 0], cols], axis=1)
                scale = np.abs(K).max() * (np.abs(f).max() + np.abs(mult).max() + abs(s))
                assert np.abs(K.T @ r).max() < 1e-13 * scale
                assert np.array_equal(f[cn <= 0], fk[cn <= 0])
