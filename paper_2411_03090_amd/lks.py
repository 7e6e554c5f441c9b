"""ctypes binding of the C ABI in include/lks.h.

Argument marshalling only: every step of the LKS/ALKS path runs in the HIP
library ``liblks.so`` built from ``csrc/``. There is no fallback: if the
library is missing this module raises at import time. PyTorch provides the
device memory (the workspace and the gamma / dJ/dgamma tensors) and the
stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblks.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first (__graft_entry__.build())")

# PyTorch ships its own HIP runtime under the same soname as the system one
# (libamdhip64.so.7). Loading torch first makes the library bind to the
# runtime torch already uses, so device memory and streams are shared by one
# runtime in the process whatever the import order of the caller.
try:
    import torch  # noqa: F401
except ImportError:  # CPU-only use: validation and planning need no runtime
    pass

_lib = ctypes.CDLL(LIB_PATH)

# status codes
LKS_OK = 0
LKS_E_INVALID = 1
LKS_E_NOMEM = 2
LKS_E_HIP = 3
LKS_E_STATE = 4
LKS_E_DIVERGED = 5
LKS_E_UNSUPPORTED = 6
LKS_D2Q9, LKS_D3Q19 = 0, 1
LKS_FP64, LKS_FP32DEV, LKS_MIXED = 0, 1, 2
_PRECISION = {"fp64": LKS_FP64, "fp32": LKS_FP32DEV, "mixed": LKS_MIXED}
LKS_OBJ_PRESSURE_DROP, LKS_OBJ_HEAT, LKS_OBJ_HEAT_EXCHANGE, LKS_OBJ_HEAT_SINK = 0, 1, 2, 3
LKS_STEADY, LKS_UNSTEADY = 0, 1
LKS_ADJ_PAPER, LKS_ADJ_EXACT = 0, 1
LKS_CKPT_AUTO, LKS_CKPT_TWO_LEVEL, LKS_CKPT_BINOMIAL = 0, 1, 2
_CKPT = {"auto": LKS_CKPT_AUTO, "two_level": LKS_CKPT_TWO_LEVEL, "binomial": LKS_CKPT_BINOMIAL}
FIELDS = {"drho": 0, "ux": 1, "uy": 2, "T": 3,
          "adj_rho": 4, "adj_vx": 5, "adj_vy": 6, "adj_theta": 7,
          "uz": 8, "adj_vz": 9}

EXPORTED = ("lks_create", "lks_workspace_size", "lks_bind_workspace", "lks_forward",
            "lks_advance", "lks_objective", "alks_backward", "alks_advance",
            "lks_read_field", "lks_write_field", "lks_memory_report", "lks_strerror",
            "lks_last_error", "lks_destroy", "lks_batch_create", "lks_batch_workspace_size",
            "lks_batch_bind_workspace", "lks_batch_run", "lks_batch_read_field",
            "lks_batch_last_error", "lks_batch_destroy", "lks_autotune",
            "lks_batch_autotune", "lks_set_tile_rows", "lks_set_steps_per_launch",
            "lks_launch_shape", "lks_batch_set_tile_rows", "lks_set_adjoint_mode",
            "lks_set_checkpointing", "lks_checkpoint_info", "lks_gradient_status",
            "lks_bind_static_workspace", "lks_batch_set_memory_budget",
            "lks_batch_set_adjoint_mode", "lks_batch_checkpoint_info",
            "lks_set_fused_adjoint")

# LKS_STATIC_WORKSPACE_BYTES of lks.h
STATIC_WORKSPACE_BYTES = 64 * 1024 * 1024


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("lattice", ctypes.c_int), ("precision", ctypes.c_int),
                ("periodic", ctypes.c_int)]


class Phys(ctypes.Structure):
    _fields_ = [("nu", ctypes.c_double), ("Pr", ctypes.c_double),
                ("alpha_max", ctypes.c_double), ("q_alpha", ctypes.c_double),
                ("Ks_over_Kf", ctypes.c_double), ("q_K", ctypes.c_double),
                ("thermal", ctypes.c_int), ("gbeta", ctypes.c_double * 3),
                ("T_ref", ctypes.c_double), ("beta_max", ctypes.c_double),
                ("q_beta", ctypes.c_double)]


class BC(ctypes.Structure):
    _fields_ = [("node_class", ctypes.POINTER(ctypes.c_uint8)),
                ("u_bar", ctypes.POINTER(ctypes.c_double)),
                ("T_bar", ctypes.POINTER(ctypes.c_double)),
                ("u_factor", ctypes.POINTER(ctypes.c_double)),
                ("n_factor", ctypes.c_int), ("rho_out", ctypes.c_double),
                ("objective", ctypes.c_int), ("mode", ctypes.c_int),
                ("n_steps", ctypes.c_int)]


_vp = ctypes.c_void_p
_st = ctypes.c_int
_lib.lks_create.argtypes = [ctypes.POINTER(Grid), ctypes.POINTER(Phys), ctypes.POINTER(BC),
                            ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
_lib.lks_create.restype = _st
_lib.lks_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.lks_workspace_size.restype = _st
_lib.lks_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.lks_bind_workspace.restype = _st
_lib.lks_bind_static_workspace.argtypes = [_vp]
_lib.lks_bind_static_workspace.restype = _st
_lib.lks_forward.argtypes = [_vp, _vp, ctypes.c_int]
_lib.lks_forward.restype = _st
_lib.lks_advance.argtypes = [_vp, _vp, ctypes.c_int]
_lib.lks_advance.restype = _st
_lib.lks_objective.argtypes = [_vp, ctypes.POINTER(ctypes.c_double)]
_lib.lks_objective.restype = _st
_lib.alks_backward.argtypes = [_vp, ctypes.c_double, ctypes.c_int, _vp]
_lib.alks_backward.restype = _st
_lib.alks_advance.argtypes = [_vp, ctypes.c_double, ctypes.c_int, _vp]
_lib.alks_advance.restype = _st
_lib.lks_read_field.argtypes = [_vp, ctypes.c_int, _vp]
_lib.lks_read_field.restype = _st
_lib.lks_write_field.argtypes = [_vp, ctypes.c_int, _vp]
_lib.lks_write_field.restype = _st
_lib.lks_memory_report.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t),
                                   ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_int)]
_lib.lks_memory_report.restype = _st
_lib.lks_strerror.argtypes = [ctypes.c_int]
_lib.lks_strerror.restype = ctypes.c_char_p
_lib.lks_last_error.argtypes = [_vp]
_lib.lks_last_error.restype = ctypes.c_char_p
_lib.lks_destroy.argtypes = [_vp]
_lib.lks_destroy.restype = None
_lib.lks_batch_create.argtypes = [ctypes.c_int, ctypes.POINTER(Grid), ctypes.POINTER(Phys),
                                  ctypes.POINTER(BC), _vp, ctypes.POINTER(_vp)]
_lib.lks_batch_create.restype = _st
_lib.lks_batch_workspace_size.argtypes = [_vp, ctypes.POINTER(ctypes.c_size_t)]
_lib.lks_batch_workspace_size.restype = _st
_lib.lks_batch_bind_workspace.argtypes = [_vp, _vp, ctypes.c_size_t]
_lib.lks_batch_bind_workspace.restype = _st
_lib.lks_batch_run.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_int,
                               ctypes.c_double, ctypes.POINTER(_vp),
                               ctypes.POINTER(ctypes.c_double), ctypes.c_int]
_lib.lks_batch_run.restype = _st
_lib.lks_batch_read_field.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _vp]
_lib.lks_batch_read_field.restype = _st
_lib.lks_batch_last_error.argtypes = [_vp]
_lib.lks_batch_last_error.restype = ctypes.c_char_p
_lib.lks_autotune.argtypes = [_vp, _vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
_lib.lks_autotune.restype = _st
_lib.lks_batch_autotune.argtypes = [_vp, ctypes.POINTER(_vp), ctypes.c_int, ctypes.POINTER(_vp),
                                    ctypes.POINTER(ctypes.c_int)]
_lib.lks_batch_autotune.restype = _st
_lib.lks_set_tile_rows.argtypes = [_vp, ctypes.c_int]
_lib.lks_set_tile_rows.restype = _st
_lib.lks_set_steps_per_launch.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
_lib.lks_set_steps_per_launch.restype = _st
_lib.lks_launch_shape.argtypes = [_vp] + [ctypes.POINTER(ctypes.c_int)] * 3
_lib.lks_launch_shape.restype = _st
_lib.lks_set_adjoint_mode.argtypes = [_vp, ctypes.c_int]
_lib.lks_set_adjoint_mode.restype = _st
_lib.lks_set_fused_adjoint.argtypes = [_vp, ctypes.c_int]
_lib.lks_set_fused_adjoint.restype = _st
_lib.lks_set_checkpointing.argtypes = [_vp, ctypes.c_int, ctypes.c_int]
_lib.lks_set_checkpointing.restype = _st
_lib.lks_checkpoint_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_longlong)]
_lib.lks_checkpoint_info.restype = _st
_lib.lks_gradient_status.argtypes = [_vp]
_lib.lks_gradient_status.restype = _st
_lib.lks_batch_set_tile_rows.argtypes = [_vp, ctypes.c_int]
_lib.lks_batch_set_tile_rows.restype = _st
_lib.lks_batch_destroy.argtypes = [_vp]
_lib.lks_batch_destroy.restype = None
_lib.lks_batch_set_memory_budget.argtypes = [_vp, ctypes.c_size_t]
_lib.lks_batch_set_memory_budget.restype = _st
_lib.lks_batch_set_adjoint_mode.argtypes = [_vp, ctypes.c_int]
_lib.lks_batch_set_adjoint_mode.restype = _st
_lib.lks_batch_checkpoint_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int),
                                           ctypes.POINTER(ctypes.c_longlong),
                                           ctypes.POINTER(ctypes.c_size_t)]
_lib.lks_batch_checkpoint_info.restype = _st


class LKSError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_lib.lks_strerror(status).decode()}: {msg}")
        self.status = status


def lib():
    return _lib


def _check(status, ctx=None):
    if status != LKS_OK:
        raise LKSError(status, _lib.lks_last_error(ctx).decode())


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class LKS:
    """One forward/adjoint problem bound to a device workspace.

    ``wl`` is a workloads.Workload (D2Q9) or workloads.Workload3 (D3Q19).
    ``precision`` is "fp64", "fp32" or "mixed" (steady D2Q9: FP64 forward,
    FP32 adjoint). ``mem_budget`` bounds the unsteady
    trajectory storage (bytes, 0 = none). ``checkpointing`` is None (automatic)
    or (scheme, slots) with scheme "auto", "two_level" or "binomial"; see
    lks_set_checkpointing.
    """

    def __init__(self, wl, precision="fp64", mem_budget=0, device=None, stream=None,
                 bind=True, checkpointing=None):
        self.wl = wl
        nz = getattr(wl, "nz", 1)
        self.d3 = nz > 1 or hasattr(wl, "periodic_axes")
        self.N = wl.nx * wl.ny * nz
        self._mask = np.ascontiguousarray(wl.mask, dtype=np.uint8).reshape(-1)
        self._ubar = np.ascontiguousarray(wl.ubar, dtype=np.float64).reshape(-1)
        self._Tbar = np.ascontiguousarray(wl.Tbar, dtype=np.float64).reshape(-1)
        self._ufac = np.ascontiguousarray(wl.ufac, dtype=np.float64).reshape(-1)
        if precision not in _PRECISION:
            raise ValueError(f"precision must be one of {sorted(_PRECISION)}")
        prec = _PRECISION[precision]
        if self.d3:
            self.grid = Grid(wl.nx, wl.ny, nz, LKS_D3Q19, prec, int(wl.periodic_axes))
        else:
            self.grid = Grid(wl.nx, wl.ny, 1, LKS_D2Q9, prec, int(wl.periodic))
        gb = [float(v) for v in getattr(wl, "gbeta", (0.0, 0.0))] + [0.0, 0.0]
        self.phys = Phys(wl.nu, wl.Pr, wl.alpha_max, wl.q_alpha, wl.Ks_over_Kf, wl.q_K,
                         int(wl.thermal), (ctypes.c_double * 3)(*gb[:3]),
                         float(getattr(wl, "T_ref", 0.0)),
                         float(getattr(wl, "beta_max", 0.0)),
                         float(getattr(wl, "q_beta", 0.1)))
        self.bc = BC(self._mask.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                     _dptr(self._ubar), _dptr(self._Tbar), _dptr(self._ufac),
                     len(self._ufac), wl.rho_out, wl.objective, wl.mode,
                     wl.n_fwd if wl.mode == LKS_UNSTEADY else 0)
        self.device = device
        if bind and stream is None:
            import torch
            stream = torch.cuda.current_stream(torch.device(device or "cuda")).cuda_stream
        self.stream = stream
        self.workspace = None
        self.ctx = _vp()
        _check(_lib.lks_create(ctypes.byref(self.grid), ctypes.byref(self.phys),
                               ctypes.byref(self.bc), ctypes.c_size_t(int(mem_budget)),
                               _vp(stream or 0), ctypes.byref(self.ctx)))
        mode = getattr(wl, "adjoint_mode", "paper")
        if mode != "paper":
            self.set_adjoint_mode(mode)
        if checkpointing is not None:
            self.set_checkpointing(*checkpointing)
        if bind:
            self.bind()

    # -- workspace -------------------------------------------------------
    def workspace_size(self):
        n = ctypes.c_size_t()
        _check(_lib.lks_workspace_size(self.ctx, ctypes.byref(n)), self.ctx)
        return n.value

    def bind_static(self):
        """Bind the library's static per-device workspace array (no device
        allocation; see lks_bind_static_workspace)."""
        self.workspace = None
        _check(_lib.lks_bind_static_workspace(self.ctx), self.ctx)

    def bind(self):
        """Allocate the workspace as a torch tensor and hand it to the library."""
        import torch
        n = self.workspace_size()
        self.workspace = torch.empty(n + 256, dtype=torch.uint8,
                                     device=torch.device(self.device or "cuda"))
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _check(_lib.lks_bind_workspace(self.ctx, _vp(aligned), ctypes.c_size_t(n)), self.ctx)

    # -- calls -----------------------------------------------------------
    def forward(self, gamma, steps=None):
        steps = self.wl.n_fwd if steps is None else steps
        _check(_lib.lks_forward(self.ctx, _vp(gamma.data_ptr()), int(steps)), self.ctx)

    def advance(self, gamma, steps):
        _check(_lib.lks_advance(self.ctx, _vp(gamma.data_ptr()), int(steps)), self.ctx)

    def objective(self):
        J = ctypes.c_double()
        _check(_lib.lks_objective(self.ctx, ctypes.byref(J)), self.ctx)
        return J.value

    def backward(self, seed, out, adj_steps=None):
        adj_steps = self.wl.n_adj if adj_steps is None else adj_steps
        _check(_lib.alks_backward(self.ctx, float(seed), int(adj_steps), _vp(out.data_ptr())),
               self.ctx)

    def adjoint_advance(self, seed, steps, out=None):
        _check(_lib.alks_advance(self.ctx, float(seed), int(steps),
                                 _vp(out.data_ptr() if out is not None else 0)), self.ctx)

    def read(self, name, out=None):
        import torch
        if out is None:
            out = torch.empty(self.N, dtype=torch.float64,
                              device=torch.device(self.device or "cuda"))
        _check(_lib.lks_read_field(self.ctx, FIELDS[name], _vp(out.data_ptr())), self.ctx)
        return out

    def write(self, name, t):
        _check(_lib.lks_write_field(self.ctx, FIELDS[name], _vp(t.data_ptr())), self.ctx)

    def autotune(self, gamma, steps=200):
        """Pick the fastest tile height; returns it."""
        ty = ctypes.c_int()
        _check(_lib.lks_autotune(self.ctx, _vp(gamma.data_ptr()), int(steps), ctypes.byref(ty)),
               self.ctx)
        return ty.value

    def set_tile_rows(self, ty):
        _check(_lib.lks_set_tile_rows(self.ctx, int(ty)), self.ctx)

    def set_steps_per_launch(self, forward, adjoint=None):
        adjoint = forward if adjoint is None else adjoint
        _check(_lib.lks_set_steps_per_launch(self.ctx, int(forward), int(adjoint)), self.ctx)

    def set_adjoint_mode(self, mode):
        """"paper" (the ALKS of Sec. 2.5) or "exact" (the transpose of the
        discrete Brinkman step); see lks_set_adjoint_mode."""
        code = {"paper": LKS_ADJ_PAPER, "exact": LKS_ADJ_EXACT}[mode]
        _check(_lib.lks_set_adjoint_mode(self.ctx, code), self.ctx)

    def set_fused_adjoint(self, fused):
        """D3Q19: the ALKS step as one z-marching kernel (True) or as the
        pull, face and update passes (False); see lks_set_fused_adjoint."""
        _check(_lib.lks_set_fused_adjoint(self.ctx, int(bool(fused))), self.ctx)

    def gradient_status(self):
        """Raise LKSError (LKS_E_DIVERGED) if the last forward state or
        gradient is non-finite (synchronises the stream)."""
        _check(_lib.lks_gradient_status(self.ctx), self.ctx)

    def set_checkpointing(self, scheme, slots=0):
        """Plan the unsteady checkpoints before binding (see
        lks_set_checkpointing)."""
        _check(_lib.lks_set_checkpointing(self.ctx, _CKPT[scheme], int(slots)), self.ctx)

    def set_memory_budget(self, nbytes):
        """Device bytes for the whole batch, before binding (unsteady
        batches plan their checkpoint interval from it)."""
        _bcheck(_lib.lks_batch_set_memory_budget(self.b, ctypes.c_size_t(int(nbytes))), self.b)

    def checkpoint_info(self):
        """{"scheme": "two_level" | "binomial" | None, "count": K or snapshots,
        "replay_steps": forward steps one adjoint sweep recomputes}."""
        sc, n, r = ctypes.c_int(), ctypes.c_int(), ctypes.c_longlong()
        _check(_lib.lks_checkpoint_info(self.ctx, ctypes.byref(sc), ctypes.byref(n),
                                        ctypes.byref(r)), self.ctx)
        name = {LKS_CKPT_TWO_LEVEL: "two_level", LKS_CKPT_BINOMIAL: "binomial"}.get(sc.value)
        return {"scheme": name, "count": n.value, "replay_steps": r.value}

    def launch_shape(self):
        """(tile rows, forward steps per launch, adjoint steps per launch)."""
        ty, sf, sa = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(_lib.lks_launch_shape(self.ctx, ctypes.byref(ty), ctypes.byref(sf),
                                     ctypes.byref(sa)), self.ctx)
        return ty.value, sf.value, sa.value

    def memory_report(self):
        a, b, k = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_int()
        _check(_lib.lks_memory_report(self.ctx, ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(k)), self.ctx)
        return {"ckpt_bytes": a.value, "state_bytes": b.value, "K": k.value}

    def close(self):
        if self.ctx:
            _lib.lks_destroy(self.ctx)
            self.ctx = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass




def _bcheck(status, b=None):
    if status != LKS_OK:
        raise LKSError(status, _lib.lks_batch_last_error(b).decode())


class Batch:
    """Many independent designs advanced together: one kernel launch per step
    for all designs, the step sequence replayed as a HIP graph. Steady
    pressure-drop designs, or unsteady designs sharing one horizon, whose
    sweeps are checkpointed with one interval chosen for mem_budget bytes
    (0: every level kept)."""

    def __init__(self, workloads, precision="fp32", device=None, stream=None, bind=True,
                 mem_budget=0, adjoint_mode=None):
        self.wls = list(workloads)
        self.n = len(self.wls)
        self._keep = [LKS(w, precision=precision, bind=False, stream=0) for w in self.wls]
        self.grids = (Grid * self.n)(*[k.grid for k in self._keep])
        self.phys = (Phys * self.n)(*[k.phys for k in self._keep])
        self.bcs = (BC * self.n)(*[k.bc for k in self._keep])
        self.device = device
        if bind and stream is None:
            import torch
            stream = torch.cuda.current_stream(torch.device(device or "cuda")).cuda_stream
        self.stream = stream
        self.b = _vp()
        _bcheck(_lib.lks_batch_create(self.n, self.grids, self.phys, self.bcs, _vp(stream or 0),
                                      ctypes.byref(self.b)))
        if mem_budget:
            self.set_memory_budget(mem_budget)
        if adjoint_mode is None:
            adjoint_mode = getattr(self.wls[0], "adjoint_mode", "paper")
        if adjoint_mode != "paper":
            code = {"paper": LKS_ADJ_PAPER, "exact": LKS_ADJ_EXACT}[adjoint_mode]
            _bcheck(_lib.lks_batch_set_adjoint_mode(self.b, code), self.b)
        self.workspace = None
        if bind:
            self.bind()

    def workspace_size(self):
        n = ctypes.c_size_t()
        _bcheck(_lib.lks_batch_workspace_size(self.b, ctypes.byref(n)), self.b)
        return n.value

    def bind(self):
        import torch
        n = self.workspace_size()
        self.workspace = torch.empty(n + 256, dtype=torch.uint8,
                                     device=torch.device(self.device or "cuda"))
        aligned = (self.workspace.data_ptr() + 255) & ~255
        _bcheck(_lib.lks_batch_bind_workspace(self.b, _vp(aligned), ctypes.c_size_t(n)), self.b)

    def run(self, gammas, outs, n_fwd, n_adj, seed=1.0, graph=True):
        g = (_vp * self.n)(*[t.data_ptr() for t in gammas])
        o = (_vp * self.n)(*[t.data_ptr() for t in outs])
        J = (ctypes.c_double * self.n)()
        _bcheck(_lib.lks_batch_run(self.b, g, int(n_fwd), int(n_adj), float(seed), o, J,
                                   int(bool(graph))), self.b)
        return list(J)

    def set_memory_budget(self, nbytes):
        """Device bytes for the whole batch, before binding (unsteady
        batches plan their checkpoint interval from it)."""
        _bcheck(_lib.lks_batch_set_memory_budget(self.b, ctypes.c_size_t(int(nbytes))), self.b)

    def checkpoint_info(self):
        """(K, replay steps, workspace bytes) of the batch's plan."""
        K, rep, ws = ctypes.c_int(), ctypes.c_longlong(), ctypes.c_size_t()
        _bcheck(_lib.lks_batch_checkpoint_info(self.b, ctypes.byref(K), ctypes.byref(rep),
                                               ctypes.byref(ws)), self.b)
        return K.value, rep.value, ws.value

    def autotune(self, gammas, scratch, steps=100):
        g = (_vp * self.n)(*[t.data_ptr() for t in gammas])
        o = (_vp * self.n)(*[t.data_ptr() for t in scratch])
        ty = ctypes.c_int()
        _bcheck(_lib.lks_batch_autotune(self.b, g, int(steps), o, ctypes.byref(ty)), self.b)
        return ty.value

    def set_tile_rows(self, ty):
        _bcheck(_lib.lks_batch_set_tile_rows(self.b, int(ty)), self.b)

    def read(self, design, name, out=None):
        import torch
        wl = self.wls[design]
        if out is None:
            out = torch.empty(wl.nx * wl.ny, dtype=torch.float64, device=self.workspace.device)
        _bcheck(_lib.lks_batch_read_field(self.b, int(design), FIELDS[name], _vp(out.data_ptr())),
                self.b)
        return out

    def close(self):
        if self.b:
            _lib.lks_batch_destroy(self.b)
            self.b = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
