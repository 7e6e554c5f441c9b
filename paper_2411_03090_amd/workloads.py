"""Seeded synthetic workloads for the LKS/ALKS path.

This module builds the *inputs* of a run -- node-class masks, design fields
gamma, prescribed boundary values and inflow time factors -- from a seed. It
holds none of the scheme's arithmetic (no equilibria, gradients, adjoints or
sensitivities), so that the FP64 oracle and the HIP library can both be fed
from it without sharing any code of the method.

Node-class byte (one per lattice node, x fastest) -- the input format of both
implementations:

    bits 0-1  flow class   0 interior (design) node, 1 prescribed velocity
                           (inlet or wall), 2 prescribed pressure (outlet),
                           3 corner
    bits 2-3  thermal      0 none/interior, 1 prescribed temperature,
                           2 prescribed heat flux (the flux into the domain
                           is the node's T_bar value; 0 is adiabatic)
    bit  4    member of the inlet set of the pressure-drop objective
    bit  5    member of the outlet set of the pressure-drop objective
    bit  6    member of the probe set of the heat-transfer objective, or of
              the heated boundary of the heat-sink objective

The geometry is the rectangle of nodes [0,nx) x [0,ny); the outer ring of
nodes is the boundary (Sec. 2.4 prescribes velocity at inlets and walls,
pressure and zero tangential velocity at outlets, temperature or heat flux
on thermal boundaries).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLOW_INTERIOR = 0
FLOW_VELOCITY = 1
FLOW_PRESSURE = 2
FLOW_CORNER = 3
THERM_NONE = 0 << 2
THERM_DIRICHLET = 1 << 2
THERM_FLUX = 2 << 2
TAG_J_INLET = 1 << 4
TAG_J_OUTLET = 1 << 5
TAG_PROBE = 1 << 6

OBJ_PRESSURE_DROP = 0
OBJ_HEAT = 1
OBJ_HEAT_EXCHANGE = 2
OBJ_HEAT_SINK = 3
MODE_STEADY = 0
MODE_UNSTEADY = 1


@dataclass
class Workload:
    """Everything a forward+adjoint run needs, as plain arrays and scalars."""
    name: str
    nx: int
    ny: int
    nu: float
    u_max: float
    alpha_max: float
    q_alpha: float
    thermal: bool
    Pr: float = 6.0
    Ks_over_Kf: float = 1.0
    q_K: float = 0.1
    rho_out: float = 1.0
    objective: int = OBJ_PRESSURE_DROP
    mode: int = MODE_STEADY
    n_fwd: int = 0
    n_adj: int = 0
    periodic: bool = False
    # "paper": the ALKS of Sec. 2.5 (u~ divided by 1 + alpha where it is
    # formed); "exact": the transpose of the discrete Brinkman step (V divided
    # by 1 + alpha at its node, sensitivity alpha' u.V / (1 + alpha))
    adjoint_mode: str = "paper"
    # Boussinesq force G = g beta (T - T_ref) (eq:boussinesqforce): the vector
    # g beta and T_ref, lattice units; zero means no force
    gbeta: tuple = (0.0, 0.0)
    T_ref: float = 0.0
    # heat source Q = beta_gamma (1 - T) (eq:heatsource) with
    # beta_gamma = beta_max q_beta (1 - gamma) / (q_beta + gamma)
    # (eq:betagamma); beta_max = 0 means no source
    beta_max: float = 0.0
    q_beta: float = 0.1
    mask: np.ndarray = field(default=None, repr=False)      # (ny, nx) uint8
    gamma: np.ndarray = field(default=None, repr=False)     # (ny, nx) f64
    ubar: np.ndarray = field(default=None, repr=False)      # (2, ny, nx) f64
    Tbar: np.ndarray = field(default=None, repr=False)      # (ny, nx) f64
    ufac: np.ndarray = field(default=None, repr=False)      # (n_fwd+1,) f64

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny


# --------------------------------------------------------------------------
# geometry
# --------------------------------------------------------------------------
def channel_mask(nx: int, ny: int, thermal: bool, probe_col: int | None = None):
    """Channel: inlet on the left column, outlet on the right column, walls
    top and bottom, corners separate. Thermal tags: inlet and bottom wall
    prescribed temperature, top wall and outlet adiabatic."""
    if nx < 4 or ny < 4:
        raise ValueError("channel needs nx, ny >= 4")
    m = np.zeros((ny, nx), np.uint8)
    m[1:-1, 0] = FLOW_VELOCITY | TAG_J_INLET
    m[1:-1, -1] = FLOW_PRESSURE | TAG_J_OUTLET
    m[0, 1:-1] = FLOW_VELOCITY
    m[-1, 1:-1] = FLOW_VELOCITY
    for j, i in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        m[j, i] = FLOW_CORNER
    if thermal:
        m[1:-1, 0] |= THERM_DIRICHLET
        m[0, 1:-1] |= THERM_DIRICHLET
        m[-1, 1:-1] |= THERM_FLUX
        m[1:-1, -1] |= THERM_FLUX
    if probe_col is not None:
        m[1:-1, probe_col] |= TAG_PROBE
    return m


def parabolic_inflow(ny: int, u_max: float):
    """u_x(j) = u_max * 4 j (H-j) / H^2 with H = ny-1 (zero at both walls)."""
    H = ny - 1
    j = np.arange(ny, dtype=np.float64)
    return u_max * 4.0 * j * (H - j) / (H * H)


def channel_boundary_values(nx: int, ny: int, u_max: float, thermal: bool,
                            T_in: float = 0.0, T_wall: float = 1.0):
    ubar = np.zeros((2, ny, nx))
    ubar[0, 1:-1, 0] = parabolic_inflow(ny, u_max)[1:-1]
    Tbar = np.zeros((ny, nx))
    if thermal:
        Tbar[1:-1, 0] = T_in
        Tbar[0, 1:-1] = T_wall
    return ubar, Tbar


# --------------------------------------------------------------------------
# design fields
# --------------------------------------------------------------------------
def gamma_uniform(nx: int, ny: int, seed: int):
    """i.i.d. uniform[0,1] design; the boundary ring is fluid (gamma = 1)."""
    g = np.random.default_rng(seed).random((ny, nx))
    _ring_to_fluid(g)
    return g


def gaussian_random_field(shape, sigma: float, seed: int):
    """White N(0,1) noise from default_rng(seed), blurred by a periodic FFT
    Gaussian of standard deviation sigma cells, normalised to unit std."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(shape)
    k = [np.fft.fftfreq(n) for n in shape]
    grids = np.meshgrid(*k, indexing="ij")
    k2 = sum(g * g for g in grids)
    kern = np.exp(-2.0 * (math.pi ** 2) * (sigma ** 2) * k2)
    z = np.real(np.fft.ifftn(np.fft.fftn(z) * kern))
    return z / z.std()


def gamma_grf(nx: int, ny: int, sigma: float, seed: int):
    """gamma = clip(0.5 + 0.5 z, 0, 1) of a smoothed Gaussian field; ring = 1."""
    z = gaussian_random_field((ny, nx), sigma, seed)
    g = np.clip(0.5 + 0.5 * z, 0.0, 1.0)
    _ring_to_fluid(g)
    return g


def _ring_to_fluid(g):
    g[0, :] = 1.0
    g[-1, :] = 1.0
    g[:, 0] = 1.0
    g[:, -1] = 1.0


# --------------------------------------------------------------------------
# time factors
# --------------------------------------------------------------------------
def oscillating_factors(n_levels: int, amp: float, period: float):
    """Inflow factor per time level n: 1 + amp * sin(2 pi n / period)."""
    n = np.arange(n_levels, dtype=np.float64)
    return 1.0 + amp * np.sin(2.0 * math.pi * n / period)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
def _steady_channel(name, nx, ny, Re, gamma, n_fwd, n_adj, nu=0.1):
    H = ny - 1
    u_max = Re * nu / H
    if u_max > 0.1:                       # keep the inflow low-Mach
        u_max = 0.1
        nu = u_max * H / Re
    mask = channel_mask(nx, ny, thermal=False)
    ubar, Tbar = channel_boundary_values(nx, ny, u_max, thermal=False)
    return Workload(name=name, nx=nx, ny=ny, nu=nu, u_max=u_max,
                    alpha_max=1e3 / Re, q_alpha=0.1, thermal=False,
                    objective=OBJ_PRESSURE_DROP, mode=MODE_STEADY,
                    n_fwd=n_fwd, n_adj=n_adj, mask=mask, gamma=gamma,
                    ubar=ubar, Tbar=Tbar, ufac=np.ones(n_fwd + 1))


def steady_channel_uniform(nx=64, ny=64, Re=10.0, seed=0, n_fwd=3000, n_adj=3000):
    """Steady non-thermal channel, gamma i.i.d. uniform (the 64x64, Re=10,
    3000+3000-step pressure-drop case at its defaults)."""
    return _steady_channel(f"steady_uniform_{nx}x{ny}_Re{Re:g}", nx, ny, Re,
                           gamma_uniform(nx, ny, seed), n_fwd, n_adj)


def steady_channel_grf(nx=512, ny=512, Re=100.0, sigma=8.0, seed=0,
                       n_fwd=40000, n_adj=40000):
    """Steady non-thermal channel, gamma from a smoothed Gaussian field (the
    512x512, Re=100, 40000+40000-step case at its defaults)."""
    return _steady_channel(f"steady_grf_{nx}x{ny}_Re{Re:g}", nx, ny, Re,
                           gamma_grf(nx, ny, sigma, seed), n_fwd, n_adj)


def unsteady_thermal_channel(nx=1024, ny=512, Re=200.0, Pr=6.0, sigma=8.0,
                             seed=0, n_steps=20000, period=5000.0, amp=0.2,
                             nu=0.1, Ks_over_Kf=2.0, q_K=0.1):
    """Unsteady forced convection: oscillating parabolic inflow at T=0,
    heated bottom wall T=1, adiabatic top wall and outlet; objective is the
    time-averaged enthalpy flux through the last interior column.

    The solid conductivity defaults to twice the fluid's: with a contrast of
    five or more (B_s well below B_f) the ALKS thermal adjoint of eq:ageq,
    whose -B div q~ - grad B . q~ is the continuous product rule rather than
    the transpose of the discrete forward, grows without bound over horizons
    of thousands of steps."""
    H = ny - 1
    u_max = Re * nu / H
    if u_max > 0.1:                       # keep the inflow low-Mach
        u_max = 0.1
        nu = u_max * H / Re
    mask = channel_mask(nx, ny, thermal=True, probe_col=nx - 2)
    ubar, Tbar = channel_boundary_values(nx, ny, u_max, thermal=True)
    return Workload(name=f"unsteady_thermal_{nx}x{ny}_Re{Re:g}", nx=nx, ny=ny,
                    nu=nu, u_max=u_max, alpha_max=1e3 / Re, q_alpha=0.1,
                    thermal=True, Pr=Pr, Ks_over_Kf=Ks_over_Kf, q_K=q_K,
                    objective=OBJ_HEAT, mode=MODE_UNSTEADY, n_fwd=n_steps,
                    n_adj=n_steps, mask=mask, gamma=gamma_grf(nx, ny, sigma, seed),
                    ubar=ubar, Tbar=Tbar,
                    ufac=oscillating_factors(n_steps + 1, amp, period))


def heat_exchanger(n=201, Re=100.0, Pr=6.0, beta_max=0.1, q_beta=0.1, sigma=8.0,
                   seed=0, n_fwd=20000, n_adj=20000, nu=0.1):
    """Steady forced-convection heat exchanger on an n x n grid: coolant
    enters at T = 0 through the middle third of the left side with a parabolic
    profile and leaves through the middle third of the right side; every other
    boundary node is a no-slip adiabatic wall. The solid generates heat
    Q = beta_gamma (1 - T) and the objective is the heat-exchange amount
    J = -sum beta_gamma (1 - T) on the final state (Sec. 3.3 at 201 x 201).

    The inlet spans nodes a..b = round(n/3)..n-1-round(n/3) and L = b - a;
    u_max = Re nu / L is capped at 0.1 with nu lowered to keep Re (the
    paper's Re = 100, nu = 0.1, L = 200/3 would put u_max at 0.15). The
    inlet and outlet nodes also carry the pressure-drop tags, for the
    pressure-drop constraint of the same problem."""
    a = int(round(n / 3.0))
    b = n - 1 - a
    L = b - a
    u_max = Re * nu / L
    if u_max > 0.1:
        u_max = 0.1
        nu = u_max * L / Re
    m = np.zeros((n, n), np.uint8)
    m[1:-1, 0] = FLOW_VELOCITY | THERM_FLUX
    m[1:-1, -1] = FLOW_VELOCITY | THERM_FLUX
    m[0, 1:-1] = FLOW_VELOCITY | THERM_FLUX
    m[-1, 1:-1] = FLOW_VELOCITY | THERM_FLUX
    m[a:b + 1, 0] = FLOW_VELOCITY | THERM_DIRICHLET | TAG_J_INLET
    m[a:b + 1, -1] = FLOW_PRESSURE | THERM_FLUX | TAG_J_OUTLET
    for j, i in ((0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1)):
        m[j, i] = FLOW_CORNER
    ubar = np.zeros((2, n, n))
    jj = np.arange(a, b + 1, dtype=np.float64)
    ubar[0, a:b + 1, 0] = u_max * 4.0 * (jj - a) * (b - jj) / float(L * L)
    Tbar = np.zeros((n, n))
    return Workload(name=f"heat_exchanger_{n}x{n}_Re{Re:g}_b{beta_max:g}", nx=n, ny=n,
                    nu=nu, u_max=u_max, alpha_max=1e3 / Re, q_alpha=0.1,
                    thermal=True, Pr=Pr, Ks_over_Kf=1.0, q_K=0.1,
                    objective=OBJ_HEAT_EXCHANGE, mode=MODE_STEADY, n_fwd=n_fwd,
                    n_adj=n_adj, beta_max=beta_max, q_beta=q_beta, mask=m,
                    gamma=gamma_grf(n, n, sigma, seed), ubar=ubar, Tbar=Tbar,
                    ufac=np.ones(n_fwd + 1))


def heat_sink(nx=141, ny=161, Ra=2e5, Pr=6.0, q0=1e-2, Ks_over_Kf=10.0, heater=0.2,
              sigma=6.0, seed=0, n_steps=50000, nu=0.1, alpha_max=10.0, n=None):
    """Transient natural-convection heat sink in a closed nx x ny cavity (Sec.
    3.4: 141 x 161 nodes and 50000 steps, as its memory table lists, with
    L = ny - 1 = 160; n gives a square n x n cavity instead): no-slip walls;
    T = 0 on the left, right and top walls; the bottom wall adiabatic except
    the heated boundary, the middle `heater` fraction of it, where the heat
    flux q0 enters; the Boussinesq force G = g beta (T - T_ref) with
    T_ref = 0 and g beta pointing up, sized by Ra = g beta dT L^3 / (nu K_f)
    with dT = 1; objective the mean temperature over the heated boundary
    averaged over levels 1..N."""
    if n is not None:
        nx = ny = n
    L = ny - 1
    Kf = nu / Pr
    gb = Ra * nu * Kf / L ** 3
    m = np.zeros((ny, nx), np.uint8)
    m[1:-1, 0] = FLOW_VELOCITY | THERM_DIRICHLET
    m[1:-1, -1] = FLOW_VELOCITY | THERM_DIRICHLET
    m[-1, 1:-1] = FLOW_VELOCITY | THERM_DIRICHLET
    m[0, 1:-1] = FLOW_VELOCITY | THERM_FLUX
    h0 = int(round(nx * (0.5 - heater / 2)))
    h1 = nx - 1 - h0
    m[0, h0:h1 + 1] |= TAG_PROBE
    for j, i in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        m[j, i] = FLOW_CORNER
    Tbar = np.zeros((ny, nx))
    Tbar[0, h0:h1 + 1] = q0
    g = gamma_grf(nx, ny, sigma, seed)
    return Workload(name=f"heat_sink_{nx}x{ny}_Ra{Ra:g}", nx=nx, ny=ny, nu=nu, u_max=0.0,
                    alpha_max=alpha_max, q_alpha=0.1, thermal=True, Pr=Pr,
                    Ks_over_Kf=Ks_over_Kf, q_K=0.1, objective=OBJ_HEAT_SINK,
                    mode=MODE_UNSTEADY, n_fwd=n_steps, n_adj=n_steps, gbeta=(0.0, gb),
                    T_ref=0.0, mask=m, gamma=g, ubar=np.zeros((2, ny, nx)), Tbar=Tbar,
                    ufac=np.ones(n_steps + 1))


def sensitivity_check_square(n=101, Re=1.0, alpha_max=1.0, n_fwd=20000, n_adj=20000, nu=0.1):
    """The non-thermal sensitivity check of Sec. 2.6: a square of
    (n-1) x (n-1) cells (101 x 101 nodes for the paper's 100 dx) closed by
    no-slip walls, with a parabolic inflow through the middle third of the
    left side (nodes 33..67 at n = 101, the roots of the printed profile) and
    a pressure outlet on the same span of the right side; gamma = 0.1 inside
    the centred circle of radius (n-1)/6 and 0.9 elsewhere, the ring fluid;
    Re = 1 on the characteristic length (n-1)/3 with nu = 0.1. The paper does
    not print alpha_bar; it is a parameter here. The inlet and outlet nodes
    carry the pressure-drop tags."""
    H = n - 1
    a, b = int(round(H / 3.0)), int(round(2.0 * H / 3.0))
    m = np.zeros((n, n), np.uint8)
    m[1:-1, 0] = FLOW_VELOCITY
    m[1:-1, -1] = FLOW_VELOCITY
    m[0, 1:-1] = FLOW_VELOCITY
    m[-1, 1:-1] = FLOW_VELOCITY
    m[a:b + 1, 0] = FLOW_VELOCITY | TAG_J_INLET
    m[a:b + 1, -1] = FLOW_PRESSURE | TAG_J_OUTLET
    for j, i in ((0, 0), (0, n - 1), (n - 1, 0), (n - 1, n - 1)):
        m[j, i] = FLOW_CORNER
    u_max = Re * nu / (H / 3.0)
    ubar = np.zeros((2, n, n))
    jj = np.arange(a, b + 1, dtype=np.float64)
    ubar[0, a:b + 1, 0] = u_max * 4.0 * (jj - a) * (b - jj) / float((b - a) ** 2)
    g = np.full((n, n), 0.9)
    y, x = np.mgrid[0:n, 0:n]
    g[(x - H / 2.0) ** 2 + (y - H / 2.0) ** 2 <= (H / 6.0) ** 2] = 0.1
    _ring_to_fluid(g)
    return Workload(name=f"sensitivity_check_square_{n}_a{alpha_max:g}", nx=n, ny=n, nu=nu,
                    u_max=u_max, alpha_max=alpha_max, q_alpha=0.1, thermal=False,
                    objective=OBJ_PRESSURE_DROP, mode=MODE_STEADY, n_fwd=n_fwd, n_adj=n_adj,
                    mask=m, gamma=g, ubar=ubar, Tbar=np.zeros((n, n)),
                    ufac=np.ones(n_fwd + 1))


def sensitivity_check_natural_convection(nx=141, ny=81, Ra=2e5, Pr=6.0, Ks_over_Kf=10.0,
                                         q0=1e-2, n_steps=2000, nu=0.1, alpha_max=10.0,
                                         heater=4, adjoint_mode="paper"):
    """The natural-convection sensitivity check of Sec. 2.6: a closed cavity
    of 140 x 80 cells (141 x 81 nodes), no-slip walls, prescribed temperature
    T = 0 on the left, right and top sides, the bottom side adiabatic except
    its centred `heater` cells (4 dx as printed), where the heat flux q0
    enters; gamma = 1 outside the centred design domain of 80 x 50 cells,
    0.9 inside it and 0.1 in its centred 40 x 25 core. The paper leaves the
    Rayleigh number, the conductivity ratio, alpha_bar, the horizon and the
    objective unstated; they are taken from the heat-sink problem of Sec. 3.4
    (Boussinesq force sized by Ra on L = ny - 1, K_s = 10 K_f, the mean
    temperature of the heated boundary averaged over the horizon)."""
    L = ny - 1
    Kf = nu / Pr
    gb = Ra * nu * Kf / L ** 3
    m = np.zeros((ny, nx), np.uint8)
    m[1:-1, 0] = FLOW_VELOCITY | THERM_DIRICHLET
    m[1:-1, -1] = FLOW_VELOCITY | THERM_DIRICHLET
    m[-1, 1:-1] = FLOW_VELOCITY | THERM_DIRICHLET
    m[0, 1:-1] = FLOW_VELOCITY | THERM_FLUX
    h0 = (nx - 1 - heater) // 2
    h1 = h0 + heater
    m[0, h0:h1 + 1] |= TAG_PROBE
    for j, i in ((0, 0), (0, nx - 1), (ny - 1, 0), (ny - 1, nx - 1)):
        m[j, i] = FLOW_CORNER
    Tbar = np.zeros((ny, nx))
    Tbar[0, h0:h1 + 1] = q0
    g = np.ones((ny, nx))
    dx0, dy0 = (nx - 1 - 80) // 2, (ny - 1 - 50) // 2
    g[dy0:dy0 + 51, dx0:dx0 + 81] = 0.9
    cx0, cy0 = (nx - 1 - 40) // 2, (ny - 1 - 25) // 2
    g[cy0:cy0 + 26, cx0:cx0 + 41] = 0.1
    return Workload(name=f"sensitivity_check_nc_{nx}x{ny}", nx=nx, ny=ny, nu=nu, u_max=0.0,
                    alpha_max=alpha_max, q_alpha=0.1, thermal=True, Pr=Pr,
                    Ks_over_Kf=Ks_over_Kf, q_K=0.1, objective=OBJ_HEAT_SINK,
                    mode=MODE_UNSTEADY, n_fwd=n_steps, n_adj=n_steps, gbeta=(0.0, gb),
                    T_ref=0.0, mask=m, gamma=g, ubar=np.zeros((2, ny, nx)), Tbar=Tbar,
                    ufac=np.ones(n_steps + 1), adjoint_mode=adjoint_mode)


def batch_designs(n_designs=64, sizes=(128, 192, 256, 384, 512),
                  Re_range=(10.0, 200.0), sigma=8.0, n_steps=2000):
    """Independent steady designs of uneven size: for design d, default_rng(d)
    draws the edge length and Re; gamma is a smoothed random field."""
    out = []
    for d in range(n_designs):
        rng = np.random.default_rng(d)
        L = int(rng.choice(sizes))
        Re = float(rng.uniform(*Re_range))
        w = _steady_channel(f"batch{d}_{L}_Re{Re:.1f}", L, L, Re,
                            gamma_grf(L, L, sigma, 1000 + d), n_steps, n_steps)
        out.append(w)
    return out


def batch_unsteady_designs(n_designs=64, sizes=(128, 192, 256, 384, 512),
                           Re_range=(10.0, 200.0), sigma=8.0, n_steps=2000,
                           periods=4.0, aspect=1):
    """Independent unsteady forced-convection designs of uneven size sharing
    one horizon (the thermal channel of unsteady_thermal_channel: oscillating
    inflow at T = 0, heated bottom wall, time-averaged enthalpy flux through
    the last interior column): for design d, default_rng(d) draws the edge
    length L (grid aspect*L x L) and Re; the inflow oscillates `periods`
    times over the horizon."""
    out = []
    for d in range(n_designs):
        rng = np.random.default_rng(d)
        L = int(rng.choice(sizes))
        Re = float(rng.uniform(*Re_range))
        w = unsteady_thermal_channel(aspect * L, L, Re=Re, sigma=sigma, seed=1000 + d,
                                     n_steps=n_steps, period=n_steps / periods)
        w.name = f"ubatch{d}_{aspect * L}x{L}_Re{Re:.1f}"
        out.append(w)
    return out


def periodic_box(nx, ny, nu=0.1, thermal=False, Pr=6.0):
    """Fully periodic box (no boundary nodes): used for the scheme's exact
    discrete invariants."""
    mask = np.zeros((ny, nx), np.uint8)
    return Workload(name=f"periodic_{nx}x{ny}", nx=nx, ny=ny, nu=nu, u_max=0.0,
                    alpha_max=0.0, q_alpha=0.1, thermal=thermal, Pr=Pr,
                    periodic=True, mask=mask, gamma=np.ones((ny, nx)),
                    ubar=np.zeros((2, ny, nx)), Tbar=np.zeros((ny, nx)),
                    ufac=np.ones(1))


# --------------------------------------------------------------------------
# three-dimensional (D3Q19) workloads
# --------------------------------------------------------------------------
# Arrays are (nz, ny, nx), x fastest; ubar is (3, nz, ny, nx). A node is a
# boundary node when it sits at an end of a non-periodic axis; face nodes
# (one coordinate at an end) carry flow class 1 or 2, edge and corner nodes
# (two or three) flow class 3, "copy": they take density, temperature and
# adjoint moments from the node reached by stepping inwards along y and z.
FLOW_COPY = FLOW_CORNER
TAG_SOLID = 1 << 7          # interior node that is not a design node


@dataclass
class Workload3(Workload):
    nz: int = 1
    periodic_axes: int = 0   # bit 0: x, bit 1: y, bit 2: z

    @property
    def n_nodes(self) -> int:
        return self.nx * self.ny * self.nz


def _ends3(nx, ny, nz, periodic_axes):
    """Per node, the number of coordinates at an end of a non-periodic axis."""
    c = np.zeros((nz, ny, nx), np.int32)
    for ax, n in ((2, nx), (1, ny), (0, nz)):
        a = {2: 0, 1: 1, 0: 2}[ax]
        if (periodic_axes >> a) & 1:
            continue
        sl = [slice(None)] * 3
        for e in (0, n - 1):
            sl[ax] = e
            c[tuple(sl)] += 1
    return c


def duct_mask3(nx, ny, nz, probe_col=None):
    """Duct along x: inlet face x=0 (prescribed velocity and temperature),
    outlet face x=nx-1 (pressure, adiabatic), walls y=0, y=ny-1, z=0, z=nz-1
    (no slip, adiabatic); edges and corners copy."""
    if min(nx, ny, nz) < 4:
        raise ValueError("duct needs nx, ny, nz >= 4")
    m = np.zeros((nz, ny, nx), np.uint8)
    m[1:-1, 1:-1, 0] = FLOW_VELOCITY | TAG_J_INLET | THERM_DIRICHLET
    m[1:-1, 1:-1, -1] = FLOW_PRESSURE | TAG_J_OUTLET | THERM_FLUX
    for sl in ((slice(1, -1), 0, slice(1, -1)), (slice(1, -1), -1, slice(1, -1)),
               (0, slice(1, -1), slice(1, -1)), (-1, slice(1, -1), slice(1, -1))):
        m[sl] = FLOW_VELOCITY | THERM_FLUX
    m[_ends3(nx, ny, nz, 0) >= 2] = FLOW_COPY
    if probe_col is not None:
        m[1:-1, 1:-1, probe_col] |= TAG_PROBE
    return m


def duct_inflow3(ny, nz, u_max):
    """u_x(j, l) = 16 u_max j (Hy-j) l (Hz-l) / (Hy^2 Hz^2)."""
    Hy, Hz = ny - 1, nz - 1
    j = np.arange(ny, dtype=np.float64)[None, :]
    l = np.arange(nz, dtype=np.float64)[:, None]
    return 16.0 * u_max * j * (Hy - j) * l * (Hz - l) / (Hy * Hy * Hz * Hz)


def gamma_grf3(nx, ny, nz, sigma, seed):
    """gamma = clip(0.5 + 0.5 z, 0, 1) of a smoothed 3D Gaussian field; the
    boundary nodes are fluid (gamma = 1)."""
    z = gaussian_random_field((nz, ny, nx), sigma, seed)
    g = np.clip(0.5 + 0.5 * z, 0.0, 1.0)
    g[_ends3(nx, ny, nz, 0) > 0] = 1.0
    return g


def heated_block_duct(nx=256, ny=128, nz=128, Re=100.0, Pr=0.71, sigma=6.0, seed=0,
                      n_steps=5000, nu=0.1, block=((0.25, 0.375), (0.0, 0.25),
                                                    (0.375, 0.625)), probe_col=None):
    """Unsteady forced convection in a duct past a heated solid block (the
    256x128x128, Re=100, Pr=0.71, 5000-step case at its defaults): inflow at
    T=0 with the duct profile, started from rest; the block, given as
    fractions of the domain along x, y, z (x in [64,96), y in [0,32),
    z in [48,80) at full size, resting on the y=0 wall), is a non-design solid
    (gamma = 0) held at T = 1; objective is the time-averaged enthalpy flux
    through the plane x = nx-2 (x = probe_col when given)."""
    H = ny - 1
    u_max = Re * nu / H
    if u_max > 0.1:
        u_max = 0.1
        nu = u_max * H / Re
    m = duct_mask3(nx, ny, nz, probe_col=nx - 2 if probe_col is None else probe_col)
    ubar = np.zeros((3, nz, ny, nx))
    ubar[0, 1:-1, 1:-1, 0] = duct_inflow3(ny, nz, u_max)[1:-1, 1:-1]
    Tbar = np.zeros((nz, ny, nx))
    g = gamma_grf3(nx, ny, nz, sigma, seed)
    (x0, x1), (y0, y1), (z0, z1) = [(int(round(a * n)), int(round(b * n)))
                                    for (a, b), n in zip(block, (nx, ny, nz))]
    blk = np.zeros((nz, ny, nx), bool)
    blk[z0:z1, y0:y1, x0:x1] = True
    blk &= _ends3(nx, ny, nz, 0) < 2            # edges keep their copy rule
    m[blk] = (m[blk] & ~np.uint8(12)) | THERM_DIRICHLET
    inner = blk & (_ends3(nx, ny, nz, 0) == 0)
    m[inner] |= TAG_SOLID
    g[inner] = 0.0
    Tbar[blk] = 1.0
    return Workload3(name=f"heated_block_duct_{nx}x{ny}x{nz}_Re{Re:g}", nx=nx, ny=ny, nz=nz,
                     nu=nu, u_max=u_max, alpha_max=1e3 / Re, q_alpha=0.1, thermal=True,
                     Pr=Pr, Ks_over_Kf=1.0, q_K=0.1, objective=OBJ_HEAT,
                     mode=MODE_UNSTEADY, n_fwd=n_steps, n_adj=n_steps, mask=m, gamma=g,
                     ubar=ubar, Tbar=Tbar, ufac=np.ones(n_steps + 1), periodic_axes=0)


def extrude_z(wl: Workload, nz: int) -> Workload3:
    """The two-dimensional workload repeated along a periodic z axis (z
    velocity 0); a z-invariant D3Q19 run of it reproduces the D2Q9 run."""
    rep = lambda a: np.repeat(np.asarray(a)[None], nz, axis=0)
    ubar = np.zeros((3, nz, wl.ny, wl.nx))
    ubar[0] = rep(wl.ubar[0])
    ubar[1] = rep(wl.ubar[1])
    axes = 7 if wl.periodic else 4
    return Workload3(name=f"{wl.name}_z{nz}", nx=wl.nx, ny=wl.ny, nz=nz, nu=wl.nu,
                     u_max=wl.u_max, alpha_max=wl.alpha_max, q_alpha=wl.q_alpha,
                     thermal=wl.thermal, Pr=wl.Pr, Ks_over_Kf=wl.Ks_over_Kf, q_K=wl.q_K,
                     rho_out=wl.rho_out, objective=wl.objective, mode=wl.mode,
                     n_fwd=wl.n_fwd, n_adj=wl.n_adj, periodic=wl.periodic,
                     adjoint_mode=wl.adjoint_mode,
                     mask=rep(wl.mask).astype(np.uint8), gamma=rep(wl.gamma), ubar=ubar,
                     Tbar=rep(wl.Tbar), ufac=np.array(wl.ufac, dtype=np.float64),
                     periodic_axes=axes)


def periodic_box3(nx, ny, nz, nu=0.1, thermal=False, Pr=6.0):
    """Fully periodic 3D box (no boundary nodes)."""
    return Workload3(name=f"periodic_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, nu=nu, u_max=0.0,
                     alpha_max=0.0, q_alpha=0.1, thermal=thermal, Pr=Pr, periodic=True,
                     mask=np.zeros((nz, ny, nx), np.uint8), gamma=np.ones((nz, ny, nx)),
                     ubar=np.zeros((3, nz, ny, nx)), Tbar=np.zeros((nz, ny, nx)),
                     ufac=np.ones(1), periodic_axes=7)
