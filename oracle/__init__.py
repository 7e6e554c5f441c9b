"""FP64 CPU oracle of the LKS forward scheme and its ALKS adjoint.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use this package to check and time the GPU library. The
product path never imports it. It shares no code with the GPU library; the
arithmetic lives in ``lks_oracle.c`` (D2Q9) and ``lks_oracle3d.c`` (D3Q19, driven
from ``oracle.d3``), plain C with OpenMP over nodes, and this
module only marshals arrays and runs the time loops the paper describes
(Sec. 2.7, Steps 2-5):

  * steady problems: N_f forward steps from rest, the objective on the final
    state, then N_a adjoint steps with the state frozen at the final level
    and the seed applied every step, then the sensitivity once;
  * unsteady problems: N forward steps storing (u, T) of every level (the
    paper stores the whole trajectory, Sec. 3.2 and 3.4), the objective as
    the average over levels 1..N, then the adjoint from the terminal
    condition f~ = g~ = 0 (eq:afinitial, eq:aginitial) down to level 0,
    summing the sensitivity over levels.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lks_oracle.c")
_SRC3 = os.path.join(_HERE, "lks_oracle3d.c")
_LIB = os.path.join(_HERE, "liblks_oracle.so")

FLOW_CORNER = 3
TAG_J_INLET = 16
TAG_J_OUTLET = 32
OBJ_PRESSURE_DROP = 0
OBJ_HEAT = 1
OBJ_HEAT_EXCHANGE = 2
OBJ_HEAT_SINK = 3
TAG_PROBE = 64
MODE_STEADY = 0
MODE_UNSTEADY = 1
N_ADJ_FIELDS = 9
ADJ_NAMES = ("rho", "ux", "uy", "sxx", "sxy", "syy", "T", "qx", "qy")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C99 + OpenMP)."""
    newest = max(os.path.getmtime(_SRC), os.path.getmtime(_SRC3))
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < newest:
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-std=c99", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, _SRC3, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Problem(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("periodic", ctypes.c_int), ("thermal", ctypes.c_int),
                ("nu", ctypes.c_double), ("Kf", ctypes.c_double),
                ("Ks", ctypes.c_double), ("q_K", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("q_alpha", ctypes.c_double),
                ("rho_out", ctypes.c_double),
                ("mask", ctypes.POINTER(ctypes.c_uint8)),
                ("ubar", ctypes.POINTER(ctypes.c_double)),
                ("Tbar", ctypes.POINTER(ctypes.c_double)),
                ("adj_exact", ctypes.c_int),
                ("gbeta", ctypes.c_double * 2), ("T_ref", ctypes.c_double),
                ("beta_max", ctypes.c_double), ("q_beta", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        d = ctypes.POINTER(ctypes.c_double)
        P = ctypes.POINTER(_Problem)
        dd = ctypes.POINTER(d)
        _lib.orc_coefficients.argtypes = [P, d, d, d, d, d]
        _lib.orc_init_state.argtypes = [P, ctypes.c_double, d, d, d, d]
        _lib.orc_source_coefficients.argtypes = [P, d, d, d]
        _lib.orc_lks_step.argtypes = [P, d, d, d, ctypes.c_double, d, d, d, d, d, d, d, d]
        _lib.orc_source_heat.argtypes = [P, d, d]
        _lib.orc_source_heat.restype = ctypes.c_double
        _lib.orc_pressure_drop.argtypes = [P, d]
        _lib.orc_pressure_drop.restype = ctypes.c_double
        _lib.orc_probe_heat.argtypes = [P, d, d]
        _lib.orc_probe_heat.restype = ctypes.c_double
        _lib.orc_adjoint_equilibrium.argtypes = [P, d, d, d, dd, d, d, d, d, d]
        _lib.orc_alks_step.argtypes = [P, d, d, d, d, d, d, d, d, d, dd, dd,
                                       ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, d]
        _lib.orc_probe_T.argtypes = [P, d]
        _lib.orc_probe_T.restype = ctypes.c_double
        _lib.orc_sens_add.argtypes = [P, d, d, d, d, d, d, dd, ctypes.c_double, d]
        _lib.orc_source_sens_add.argtypes = [P, d, d, d, d, d, d, d, dd, ctypes.c_double, d]
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
        _lib.orc_max_threads.restype = ctypes.c_int
        _lib.orc_boundary_fill.argtypes = [P, ctypes.c_uint8, ctypes.c_int, ctypes.c_int,
                                           ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double, d, d, d, ctypes.c_double]
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's loops."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _pp(arrs):
    arr = (ctypes.POINTER(ctypes.c_double) * len(arrs))(*[_p(a) for a in arrs])
    return ctypes.cast(arr, ctypes.POINTER(ctypes.POINTER(ctypes.c_double))), arr


class Problem:
    """Binds a workload's arrays to the C problem descriptor."""

    def __init__(self, wl):
        self.wl = wl
        self.nx, self.ny = wl.nx, wl.ny
        self.N = wl.nx * wl.ny
        self.mask = np.ascontiguousarray(wl.mask, dtype=np.uint8).reshape(-1)
        self.ubar = np.ascontiguousarray(wl.ubar, dtype=np.float64).reshape(-1)
        self.Tbar = np.ascontiguousarray(wl.Tbar, dtype=np.float64).reshape(-1)
        Kf = wl.nu / wl.Pr
        self.c = _Problem(wl.nx, wl.ny, int(wl.periodic), int(wl.thermal), wl.nu, Kf,
                          Kf * wl.Ks_over_Kf, wl.q_K, wl.alpha_max, wl.q_alpha,
                          wl.rho_out,
                          self.mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                          _p(self.ubar), _p(self.Tbar),
                          int(getattr(wl, "adjoint_mode", "paper") == "exact"),
                          (ctypes.c_double * 2)(*[float(v) for v in getattr(wl, "gbeta", (0, 0))[:2]]),
                          float(getattr(wl, "T_ref", 0.0)),
                          float(getattr(wl, "beta_max", 0.0)),
                          float(getattr(wl, "q_beta", 0.1)))
        self.ref = ctypes.byref(self.c)

    def zeros(self, k=None):
        return np.zeros(self.N) if k is None else [np.zeros(self.N) for _ in range(k)]


@dataclass
class State:
    drho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray

    def copy(self):
        return State(self.drho.copy(), self.ux.copy(), self.uy.copy(), self.T.copy())


def coefficients(pb: Problem, gamma):
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(-1)
    a, da, B, dB = pb.zeros(4)
    lib().orc_coefficients(pb.ref, _p(g), _p(a), _p(da), _p(B), _p(dB))
    return a, da, B, dB


def source_coefficients(pb: Problem, gamma):
    """(beta, beta') of the heat source eq:heatsource / eq:betagamma, or
    (None, None) when the problem has no source."""
    if not getattr(pb.wl, "beta_max", 0.0):
        return None, None
    g = np.ascontiguousarray(gamma, dtype=np.float64).reshape(-1)
    b, db = pb.zeros(2)
    lib().orc_source_coefficients(pb.ref, _p(g), _p(b), _p(db))
    return b, db


def _opt(a):
    return None if a is None else _p(a)


def init_state(pb: Problem, ufac0=1.0) -> State:
    s = State(*pb.zeros(4))
    lib().orc_init_state(pb.ref, ufac0, _p(s.drho), _p(s.ux), _p(s.uy), _p(s.T))
    return s


def lks_step(pb: Problem, alpha, B, ufac, s: State, beta=None) -> State:
    o = State(*pb.zeros(4))
    lib().orc_lks_step(pb.ref, _p(alpha), _p(B), _opt(beta), ufac, _p(s.drho), _p(s.ux), _p(s.uy),
                       _p(s.T), _p(o.drho), _p(o.ux), _p(o.uy), _p(o.T))
    return o


def pressure_drop(pb: Problem, s: State) -> float:
    return lib().orc_pressure_drop(pb.ref, _p(s.drho))


def probe_heat(pb: Problem, s: State) -> float:
    return lib().orc_probe_heat(pb.ref, _p(s.ux), _p(s.T))


def source_heat(pb: Problem, beta, s: State) -> float:
    return lib().orc_source_heat(pb.ref, _p(beta), _p(s.T))


def level_objective(pb: Problem, s: State, beta=None) -> float:
    if pb.wl.objective == OBJ_PRESSURE_DROP:
        return pressure_drop(pb, s)
    if pb.wl.objective == OBJ_HEAT_EXCHANGE:
        return source_heat(pb, beta if beta is not None else np.zeros(pb.N), s)
    if pb.wl.objective == OBJ_HEAT_SINK:
        return lib().orc_probe_T(pb.ref, _p(s.T))
    return probe_heat(pb, s)


def heated_count(pb: Problem) -> int:
    return int(np.count_nonzero(pb.mask & TAG_PROBE))


def _seeds(pb: Problem, w):
    """(seed_dp, seed_heat, seed_src, seed_bt) of one level for objective weight w."""
    o = pb.wl.objective
    return (w if o == OBJ_PRESSURE_DROP else 0.0, w if o == OBJ_HEAT else 0.0,
            w if o == OBJ_HEAT_EXCHANGE else 0.0,
            w / max(heated_count(pb), 1) if o == OBJ_HEAT_SINK else 0.0)


def adjoint_equilibrium(pb: Problem, B, ux, uy, adj, alpha=None, beta=None):
    """(V_x, V_y, Theta): the coefficients of eq:afeq / eq:ageq; with alpha,
    V divided by 1 + alpha (the propagated coefficient of the exact mode),
    and with beta as well, Theta divided by 1 + beta."""
    Vx, Vy, Th = pb.zeros(3)
    pp, keep = _pp(adj)
    a = None if alpha is None else np.ascontiguousarray(alpha, dtype=np.float64)
    lib().orc_adjoint_equilibrium(pb.ref, _p(B), _p(ux), _p(uy), pp, _p(Vx), _p(Vy),
                                  _p(Th), None if a is None else _p(a), _opt(beta))
    return Vx, Vy, Th


def alks_step(pb: Problem, alpha, B, src: State, dst: State, adj_in, seed_dp, seed_heat,
              beta=None, seed_src=0.0, seed_bt=0.0):
    out = pb.zeros(N_ADJ_FIELDS)
    work = np.zeros(3 * pb.N)
    pin, k1 = _pp(adj_in)
    pout, k2 = _pp(out)
    lib().orc_alks_step(pb.ref, _p(alpha), _p(B), _opt(beta), _p(src.ux), _p(src.uy), _p(src.T),
                        _p(dst.ux), _p(dst.uy), _p(dst.T), pin, pout, seed_dp, seed_heat,
                        seed_src, seed_bt, _p(work))
    return out


def sens_add(pb: Problem, alpha, dalpha, dB, s: State, adj, weight, sens):
    pp, keep = _pp(adj)
    lib().orc_sens_add(pb.ref, _p(alpha), _p(dalpha), _p(dB), _p(s.ux), _p(s.uy), _p(s.T),
                       pp, weight, _p(sens))


def source_sens_add(pb: Problem, alpha, B, beta, dbeta, s: State, adj, wJ, sens):
    """Heat-source part of dJ/dgamma at one level (beta'(T - 1)(w_J + T~),
    or with the propagated Theta in exact mode)."""
    pp, keep = _pp(adj)
    lib().orc_source_sens_add(pb.ref, _p(alpha), _p(B), _p(beta), _p(dbeta), _p(s.ux),
                              _p(s.uy), _p(s.T), pp, wJ, _p(sens))


def boundary_fill(pb: Problem, m, normal, Bn, Tn, u, seed_dp, fk, gk, seed_T=0.0):
    """Completed (f~, g~) at one ring node and the multipliers
    (flow pair, thermal); seed_T is dJ/dg_i of a boundary temperature
    objective at the node."""
    fk = np.ascontiguousarray(fk, dtype=np.float64).copy()
    gk = np.ascontiguousarray(gk, dtype=np.float64).copy()
    mult = np.zeros(3)
    lib().orc_boundary_fill(pb.ref, int(m), int(normal[0]), int(normal[1]), Bn, Tn,
                            float(u[0]), float(u[1]), seed_dp, _p(fk), _p(gk), _p(mult),
                            float(seed_T))
    return fk, gk, mult


# --------------------------------------------------------------------------
# drivers
# --------------------------------------------------------------------------
class CheckpointedTrajectory:
    """Levels 0..N of a forward sweep without storing them all: the states of
    levels 0, K, 2K, ... are kept, and a level between two of them is
    recomputed, together with the rest of its segment, from the checkpoint
    that starts the segment (two-level checkpointing). Indexing returns the
    same state a stored trajectory would hold. The reverse sweep asks for
    levels in decreasing order, so each segment is recomputed once; a
    checkpoint level is served from the checkpoint itself.

    step(n, s) returns the state of level n + 1 from that of level n."""

    def __init__(self, step, state0, n_steps: int, K: int, on_level=None):
        if K < 1:
            raise ValueError("checkpoint interval must be >= 1")
        self.step, self.N, self.K = step, n_steps, K
        self.ckpt = {0: state0}
        s = state0
        for n in range(n_steps):
            s = step(n, s)
            if on_level is not None:
                on_level(n + 1, s)
            if (n + 1) % K == 0:
                self.ckpt[n + 1] = s
        self.final = s
        self.replayed = 0
        self._start, self._seg = None, None

    def __len__(self):
        return self.N + 1

    def __getitem__(self, n: int):
        if n < 0 or n > self.N:
            raise IndexError(n)
        if n in self.ckpt:
            return self.ckpt[n]
        b = (n // self.K) * self.K
        if self._start != b:
            s, seg = self.ckpt[b], [self.ckpt[b]]
            for m in range(b, min(b + self.K, self.N + 1) - 1):
                s = self.step(m, s)
                seg.append(s)
            self.replayed += len(seg) - 1
            self._start, self._seg = b, seg
        return self._seg[n - b]


def forward(pb: Problem, gamma, n_steps, store=False, state0: State | None = None,
            checkpoint: int | None = None):
    """n_steps LKS steps from the level-0 state. Returns (final state, J,
    trajectory or None). Steady: J on the final state. Unsteady: J averaged
    over levels 1..n_steps. With store, the trajectory is a list of every
    level, or with checkpoint=K a CheckpointedTrajectory that keeps every
    K-th level and recomputes the others on demand."""
    wl = pb.wl
    alpha, _, B, _ = coefficients(pb, gamma)
    beta, _ = source_coefficients(pb, gamma)
    s = init_state(pb, wl.ufac[0]) if state0 is None else state0.copy()
    acc = [0.0]

    def step(n, st):
        return lks_step(pb, alpha, B, float(wl.ufac[min(n + 1, len(wl.ufac) - 1)]), st, beta)

    def on_level(n, st):
        if wl.mode == MODE_UNSTEADY:
            acc[0] += level_objective(pb, st, beta)

    if store and checkpoint is not None:
        traj = CheckpointedTrajectory(step, s, n_steps, checkpoint, on_level)
        s = traj.final
        J = acc[0] / max(n_steps, 1) if wl.mode == MODE_UNSTEADY else level_objective(pb, s, beta)
        return s, J, traj
    traj = [s] if store else None
    for n in range(n_steps):
        s = step(n, s)
        on_level(n + 1, s)
        if store:
            traj.append(s)
    acc = acc[0]
    if wl.mode == MODE_UNSTEADY:
        J = acc / max(n_steps, 1)
    else:
        J = level_objective(pb, s, beta)
    return s, J, traj


def adjoint_steady(pb: Problem, gamma, state: State, n_adj, seed=1.0):
    """n_adj ALKS steps with (u, T) frozen at `state` and the seed applied
    every step; returns (adjoint fields, dJ/dgamma)."""
    wl = pb.wl
    alpha, dalpha, B, dB = coefficients(pb, gamma)
    beta, dbeta = source_coefficients(pb, gamma)
    adj = pb.zeros(N_ADJ_FIELDS)
    sdp, sh, ss, sbt = _seeds(pb, seed)
    for _ in range(n_adj):
        adj = alks_step(pb, alpha, B, state, state, adj, sdp, sh, beta, ss, sbt)
    sens = np.zeros(pb.N)
    sens_add(pb, alpha, dalpha, dB, state, adj, 1.0, sens)
    if beta is not None:
        source_sens_add(pb, alpha, B, beta, dbeta, state, adj, ss, sens)
    return adj, sens


def adjoint_unsteady(pb: Problem, gamma, traj, seed=1.0):
    """Reverse sweep over a stored trajectory of N+1 levels; the objective is
    the average over levels 1..N, so the seed at level n >= 1 is seed/N.
    The paper's sensitivity sums levels 0..N. The exact mode pairs each term
    with the step where gamma acts: the Brinkman and source terms with the
    levels the steps produce (1..N; the initial state does not depend on
    gamma), the conductivity term B' grad T . q~ with the levels whose
    equilibria the steps use (0..N-1; at level N q~ = 0)."""
    wl = pb.wl
    N = len(traj) - 1
    alpha, dalpha, B, dB = coefficients(pb, gamma)
    beta, dbeta = source_coefficients(pb, gamma)
    adj = pb.zeros(N_ADJ_FIELDS)
    sens = np.zeros(pb.N)
    for n in range(N, -1, -1):
        w = seed / N if n >= 1 else 0.0
        sdp, sh, ss, sbt = _seeds(pb, w)
        src = traj[min(n + 1, N)]
        adj = alks_step(pb, alpha, B, src, traj[n], adj, sdp, sh, beta, ss, sbt)
        if n >= 1 or getattr(wl, "adjoint_mode", "paper") != "exact":
            sens_add(pb, alpha, dalpha, dB, traj[n], adj, 1.0, sens)
            if beta is not None:
                source_sens_add(pb, alpha, B, beta, dbeta, traj[n], adj, ss, sens)
        else:
            # exact mode, level 0: the conductivity term only
            sens_add(pb, alpha, np.zeros(pb.N), dB, traj[n], adj, 1.0, sens)
    return adj, sens


def gradient(wl, gamma=None, seed=1.0, checkpoint: int | None = None):
    """Objective and ALKS sensitivity for a workload (steady or unsteady).
    An unsteady sweep stores every level, or with checkpoint=K every K-th
    level with replay of the others."""
    pb = Problem(wl)
    g = wl.gamma if gamma is None else gamma
    if wl.mode == MODE_STEADY:
        s, J, _ = forward(pb, g, wl.n_fwd)
        adj, sens = adjoint_steady(pb, g, s, wl.n_adj, seed)
        return J, sens.reshape(wl.ny, wl.nx), s, adj
    s, J, traj = forward(pb, g, wl.n_fwd, store=True, checkpoint=checkpoint)
    adj, sens = adjoint_unsteady(pb, g, traj, seed)
    return J, sens.reshape(wl.ny, wl.nx), s, adj


def objective(wl, gamma):
    pb = Problem(wl)
    return forward(pb, gamma, wl.n_fwd)[1]
