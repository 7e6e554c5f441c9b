"""FP64 CPU oracle of the D3Q19 extension (three-dimensional LKS and ALKS).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the arithmetic is in
``lks_oracle3d.c``; this module marshals arrays and runs the same time loops
as the two-dimensional drivers (Sec. 2.7, Steps 2-5).

State arrays are flat, x fastest: drho (N), u (3 N: x, y, z blocks), T (N).
The adjoint state is 14 arrays: rho~, u~ (3), s~ (xx, xy, xz, yy, yz, zz),
T~, q~ (3).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np

from . import CheckpointedTrajectory
from . import build as _build_lib

N_ADJ3 = 14
OBJ_PRESSURE_DROP = 0
OBJ_HEAT = 1
MODE_STEADY = 0


class _Problem3(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("periodic", ctypes.c_int), ("thermal", ctypes.c_int),
                ("nu", ctypes.c_double), ("Kf", ctypes.c_double),
                ("Ks", ctypes.c_double), ("q_K", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("q_alpha", ctypes.c_double),
                ("rho_out", ctypes.c_double),
                ("mask", ctypes.POINTER(ctypes.c_uint8)),
                ("ubar", ctypes.POINTER(ctypes.c_double)),
                ("Tbar", ctypes.POINTER(ctypes.c_double)),
                ("adj_exact", ctypes.c_int)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build_lib())
        d = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Problem3)
        dd = ctypes.POINTER(d)
        c = ctypes.c_double
        _lib.orc3_coefficients.argtypes = [P, d, d, d, d, d]
        _lib.orc3_init_state.argtypes = [P, c, d, d, d]
        _lib.orc3_lks_step.argtypes = [P, d, d, c, d, d, d, d, d, d]
        _lib.orc3_pressure_drop.argtypes = [P, d]
        _lib.orc3_pressure_drop.restype = c
        _lib.orc3_probe_heat.argtypes = [P, d, d]
        _lib.orc3_probe_heat.restype = c
        _lib.orc3_adjoint_equilibrium.argtypes = [P, d, d, dd, d, d, d]
        _lib.orc3_alks_step.argtypes = [P, d, d, d, d, d, d, dd, dd, c, c, d]
        _lib.orc3_sens_add.argtypes = [P, d, d, d, d, d, dd, c, d]
        _lib.orc3_boundary_fill.argtypes = [P, ctypes.c_uint8, ctypes.c_int, ctypes.c_int,
                                            ctypes.c_int, c, c, c, c, c, c, d, d, d]
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pp(arrs):
    arr = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_p(a) for a in arrs])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))), arr


class Problem3:
    def __init__(self, wl):
        self.wl = wl
        self.N = wl.nx * wl.ny * wl.nz
        self.mask = np.ascontiguousarray(wl.mask, dtype=np.uint8).reshape(-1)
        self.ubar = np.ascontiguousarray(wl.ubar, dtype=np.float64).reshape(-1)
        self.Tbar = np.ascontiguousarray(wl.Tbar, dtype=np.float64).reshape(-1)
        Kf = wl.nu / wl.Pr
        self.c = _Problem3(wl.nx, wl.ny, wl.nz, int(wl.periodic_axes), int(wl.thermal),
                           wl.nu, Kf, Kf * wl.Ks_over_Kf, wl.q_K, wl.alpha_max, wl.q_alpha,
                           wl.rho_out,
                           self.mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                           _p(self.ubar), _p(self.Tbar),
                           int(getattr(wl, "adjoint_mode", "paper") == "exact"))
        self.ref = ctypes.byref(self.c)

    def zeros(self, k=None, width=1):
        if k is None:
            return np.zeros(width * self.N)
        return [np.zeros(width * self.N) for _ in range(k)]


@dataclass
class State3:
    drho: np.ndarray
    u: np.ndarray      # 3 N
    T: np.ndarray

    def copy(self):
        return State3(self.drho.copy(), self.u.copy(), self.T.copy())


def coefficients(pb: Problem3, gamma):
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(-1)
    a, da, B, dB = pb.zeros(4)
    lib().orc3_coefficients(pb.ref, _p(g), _p(a), _p(da), _p(B), _p(dB))
    return a, da, B, dB


def init_state(pb: Problem3, ufac0=1.0) -> State3:
    s = State3(pb.zeros(), pb.zeros(width=3), pb.zeros())
    lib().orc3_init_state(pb.ref, ufac0, _p(s.drho), _p(s.u), _p(s.T))
    return s


def lks_step(pb: Problem3, alpha, B, ufac, s: State3) -> State3:
    o = State3(pb.zeros(), pb.zeros(width=3), pb.zeros())
    lib().orc3_lks_step(pb.ref, _p(alpha), _p(B), ufac, _p(s.drho), _p(s.u), _p(s.T),
                        _p(o.drho), _p(o.u), _p(o.T))
    return o


def level_objective(pb: Problem3, s: State3) -> float:
    if pb.wl.objective == OBJ_PRESSURE_DROP:
        return lib().orc3_pressure_drop(pb.ref, _p(s.drho))
    return lib().orc3_probe_heat(pb.ref, _p(s.u), _p(s.T))


def adjoint_equilibrium(pb: Problem3, B, u, adj, alpha=None):
    """(V (3 N), Theta): the coefficients of eq:afeq / eq:ageq; with alpha,
    V divided by 1 + alpha (the propagated coefficient of the exact mode)."""
    V, Th = pb.zeros(width=3), pb.zeros()
    pp, keep = _pp(adj)
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    lib().orc3_adjoint_equilibrium(pb.ref, _p(B), _p(u), pp, _p(V), _p(Th),
                                   None if a is None else _p(a))
    return V, Th


def alks_step(pb: Problem3, alpha, B, src: State3, dst: State3, adj_in, seed_dp, seed_heat):
    out = pb.zeros(N_ADJ3)
    work = np.zeros(4 * pb.N)
    pin, k1 = _pp(adj_in)
    pout, k2 = _pp(out)
    lib().orc3_alks_step(pb.ref, _p(alpha), _p(B), _p(src.u), _p(src.T), _p(dst.u),
                         _p(dst.T), pin, pout, seed_dp, seed_heat, _p(work))
    return out


def sens_add(pb: Problem3, alpha, dalpha, dB, s: State3, adj, weight, sens):
    pp, keep = _pp(adj)
    lib().orc3_sens_add(pb.ref, _p(alpha), _p(dalpha), _p(dB), _p(s.u), _p(s.T), pp, weight,
                        _p(sens))


def boundary_fill(pb: Problem3, m, normal, Bn, Tn, u, seed_dp, fk, gk):
    """Completed (f~, g~) at one face node and the multipliers (3 flow, 1
    thermal)."""
    fk = np.ascontiguousarray(fk, dtype=np.float64).copy()
    gk = np.ascontiguousarray(gk, dtype=np.float64).copy()
    mult = np.zeros(4)
    lib().orc3_boundary_fill(pb.ref, int(m), *[int(v) for v in normal], Bn, Tn,
                             *[float(v) for v in u], seed_dp, _p(fk), _p(gk), _p(mult))
    return fk, gk, mult


def forward(pb: Problem3, gamma, n_steps, store=False, state0: State3 | None = None,
            checkpoint: int | None = None):
    """As oracle.forward: with store, every level, or with checkpoint=K a
    CheckpointedTrajectory (every K-th level kept, the others recomputed)."""
    wl = pb.wl
    alpha, _, B, _ = coefficients(pb, gamma)
    s = init_state(pb, wl.ufac[0]) if state0 is None else state0.copy()
    acc = [0.0]

    def step(n, st):
        return lks_step(pb, alpha, B, float(wl.ufac[min(n + 1, len(wl.ufac) - 1)]), st)

    def on_level(n, st):
        if wl.mode != MODE_STEADY:
            acc[0] += level_objective(pb, st)

    if store and checkpoint is not None:
        traj = CheckpointedTrajectory(step, s, n_steps, checkpoint, on_level)
        s = traj.final
    else:
        traj = [s] if store else None
        for n in range(n_steps):
            s = step(n, s)
            on_level(n + 1, s)
            if store:
                traj.append(s)
    J = acc[0] / max(n_steps, 1) if wl.mode != MODE_STEADY else level_objective(pb, s)
    return s, J, traj


def adjoint_steady(pb: Problem3, gamma, state: State3, n_adj, seed=1.0):
    wl = pb.wl
    alpha, dalpha, B, dB = coefficients(pb, gamma)
    adj = pb.zeros(N_ADJ3)
    sdp = seed if wl.objective == OBJ_PRESSURE_DROP else 0.0
    sh = seed if wl.objective == OBJ_HEAT else 0.0
    for _ in range(n_adj):
        adj = alks_step(pb, alpha, B, state, state, adj, sdp, sh)
    sens = np.zeros(pb.N)
    sens_add(pb, alpha, dalpha, dB, state, adj, 1.0, sens)
    return adj, sens


def adjoint_unsteady(pb: Problem3, gamma, traj, seed=1.0):
    """Reverse sweep over a stored trajectory of N+1 levels; the seed at
    level n >= 1 is seed/N (time average over levels 1..N). In exact mode the
    Brinkman term sums levels 1..N and the conductivity term levels 0..N-1
    (see oracle.adjoint_unsteady)."""
    wl = pb.wl
    N = len(traj) - 1
    alpha, dalpha, B, dB = coefficients(pb, gamma)
    adj = pb.zeros(N_ADJ3)
    sens = np.zeros(pb.N)
    for n in range(N, -1, -1):
        w = seed / N if n >= 1 else 0.0
        sdp = w if wl.objective == OBJ_PRESSURE_DROP else 0.0
        sh = w if wl.objective == OBJ_HEAT else 0.0
        adj = alks_step(pb, alpha, B, traj[min(n + 1, N)], traj[n], adj, sdp, sh)
        if n >= 1 or getattr(wl, "adjoint_mode", "paper") != "exact":
            sens_add(pb, alpha, dalpha, dB, traj[n], adj, 1.0, sens)
        else:
            sens_add(pb, alpha, np.zeros(pb.N), dB, traj[n], adj, 1.0, sens)
    return adj, sens


def gradient(wl, gamma=None, seed=1.0, checkpoint: int | None = None):
    pb = Problem3(wl)
    g = wl.gamma if gamma is None else gamma
    shape = (wl.nz, wl.ny, wl.nx)
    if wl.mode == MODE_STEADY:
        s, J, _ = forward(pb, g, wl.n_fwd)
        adj, sens = adjoint_steady(pb, g, s, wl.n_adj, seed)
        return J, sens.reshape(shape), s, adj
    s, J, traj = forward(pb, g, wl.n_fwd, store=True, checkpoint=checkpoint)
    adj, sens = adjoint_unsteady(pb, g, traj, seed)
    return J, sens.reshape(shape), s, adj


def objective(wl, gamma):
    return forward(Problem3(wl), gamma, wl.n_fwd)[1]
