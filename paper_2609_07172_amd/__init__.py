"""Python binding of the cylpoisson C ABI (``include/cylpoisson.h``).

Argument marshalling only: every step of the solve runs in the HIP library
``libcylpoisson.so`` built from ``csrc/``.  There is no fallback; if the
library is missing, every call raises.  PyTorch provides device memory and
streams (tensors are passed by ``data_ptr()``, streams by handle).

The functions carry the C names without the ``cylpoisson_`` prefix; ``Plan``
wraps a plan handle.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch  # imported first: the library then binds to the HIP runtime torch loaded

__all__ = [
    "OK", "NOT_CONVERGED", "EINVAL", "ENOMEM", "EHIP", "ENONFINITE", "EDEVICE",
    "CylPoissonError", "library", "library_path", "plan_create", "plan_destroy",
    "plan_set_option", "solve", "solve_planes", "apply", "dft_forward", "dft_inverse",
    "get_stats", "get_info", "last_error", "last_status", "solve_static", "status_string", "Plan", "EXPORTED_SYMBOLS",
    "plan_get_option", "autotune", "solve_batch", "solve_plans", "Net", "plan_create_mesh",
    "VERTEX", "CELL",
]

OK, NOT_CONVERGED = 0, 1
EINVAL, ENOMEM, EHIP, ENONFINITE, EDEVICE = -1, -2, -3, -4, -5
VERTEX, CELL = 0, 1  # mesh layouts of cylpoisson_plan_create_mesh
MAX_HISTORY = 64
MAX_LEVELS = 24
KERNEL_CLASSES = ("dft_forward", "dft_inverse", "fine_down", "fine_up", "coarse_levels", "other", "fine_merged")

EXPORTED_SYMBOLS = (
    "cylpoisson_plan_create", "cylpoisson_plan_create_mesh", "cylpoisson_plan_destroy",
    "cylpoisson_plan_set_option",
    "cylpoisson_solve", "cylpoisson_solve_static", "cylpoisson_get_stats", "cylpoisson_get_info", "cylpoisson_apply",
    "cylpoisson_dft_forward", "cylpoisson_dft_inverse", "cylpoisson_solve_planes",
    "cylpoisson_last_error", "cylpoisson_last_status", "cylpoisson_status_string", "cylpoisson_plan_get_option",
    "cylpoisson_autotune", "cylpoisson_solve_batch", "cylpoisson_nn_create", "cylpoisson_nn_destroy",
    "cylpoisson_nn_weight_count", "cylpoisson_nn_get_weights", "cylpoisson_nn_set_weights",
    "cylpoisson_nn_get_grads", "cylpoisson_nn_forward", "cylpoisson_nn_loss_grad", "cylpoisson_nn_adam_step",
    "cylpoisson_nn_collect", "cylpoisson_nn_patch_count", "cylpoisson_nn_train", "cylpoisson_plan_set_net",
)

_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libcylpoisson.so")


class BC(ctypes.Structure):
    _fields_ = [("phi_r_in", ctypes.c_double), ("phi_r_out", ctypes.c_double),
                ("phi_z0", ctypes.c_double), ("phi_zL", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("cycles", ctypes.c_int), ("checks", ctypes.c_int),
                ("n_history", ctypes.c_int), ("rel_residual", ctypes.c_double),
                ("initial_residual_norm", ctypes.c_double),
                ("rel_residual_history", ctypes.c_double * MAX_HISTORY),
                ("kernel_launches", ctypes.c_int * len(KERNEL_CLASSES)),
                ("kernel_ms", ctypes.c_double * len(KERNEL_CLASSES)),
                ("refinements", ctypes.c_int), ("frozen_planes", ctypes.c_int),
                ("krylov_iterations", ctypes.c_int), ("learned_fallback", ctypes.c_int),
                ("vcycle_rate", ctypes.c_double), ("learned_rate", ctypes.c_double)]

    def as_dict(self) -> dict:
        hist = [self.rel_residual_history[i] for i in range(min(self.n_history, MAX_HISTORY))]
        return {"status": self.status, "cycles": self.cycles, "checks": self.checks,
                "rel_residual": self.rel_residual,
                "initial_residual_norm": self.initial_residual_norm,
                "history": [None if math.isnan(h) else h for h in hist],
                "kernel_launches": dict(zip(KERNEL_CLASSES, list(self.kernel_launches))),
                "kernel_ms": dict(zip(KERNEL_CLASSES, list(self.kernel_ms))),
                "refinements": self.refinements, "frozen_planes": self.frozen_planes,
                "krylov_iterations": self.krylov_iterations, "learned_fallback": self.learned_fallback,
                "vcycle_rate": self.vcycle_rate, "learned_rate": self.learned_rate}


class Info(ctypes.Structure):
    _fields_ = [("nr", ctypes.c_int), ("ntheta", ctypes.c_int), ("nz", ctypes.c_int),
                ("levels", ctypes.c_int), ("level_nr", ctypes.c_int * MAX_LEVELS),
                ("level_nz", ctypes.c_int * MAX_LEVELS), ("coarse_unknowns", ctypes.c_int),
                ("bottom_level", ctypes.c_int),
                ("workspace_bytes", ctypes.c_longlong), ("device", ctypes.c_int),
                ("fused_levels", ctypes.c_int), ("layout", ctypes.c_int), ("uniform", ctypes.c_int),
                ("direct_level", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {"nr": self.nr, "ntheta": self.ntheta, "nz": self.nz, "levels": self.levels,
                "level_shapes": [(self.level_nr[i], self.level_nz[i]) for i in range(self.levels)],
                "coarse_unknowns": self.coarse_unknowns, "bottom_level": self.bottom_level,
                "workspace_bytes": self.workspace_bytes, "device": self.device,
                "fused_levels": self.fused_levels, "layout": self.layout, "uniform": self.uniform,
                "direct_level": self.direct_level}


class CylPoissonError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{status_string(status)} ({status}): {message}")
        self.status = status


_lib = None


def library() -> ctypes.CDLL:
    """Load ``libcylpoisson.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(library_path):
        raise RuntimeError(f"HIP library not built: {library_path} is missing "
                           "(run __graft_entry__.build())")
    L = ctypes.CDLL(library_path)
    vp, dp, i, d = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_double
    L.cylpoisson_plan_create.restype = vp
    L.cylpoisson_plan_create.argtypes = [i, i, i, d, d, d, ctypes.POINTER(BC)]
    L.cylpoisson_plan_destroy.restype = None
    L.cylpoisson_plan_create_mesh.restype = vp
    L.cylpoisson_plan_create_mesh.argtypes = [i, i, i, ctypes.POINTER(d), ctypes.POINTER(d), i, ctypes.POINTER(BC)]
    L.cylpoisson_plan_destroy.argtypes = [vp]
    L.cylpoisson_plan_set_option.restype = i
    L.cylpoisson_plan_set_option.argtypes = [vp, ctypes.c_char_p, d]
    for name in ("cylpoisson_solve", "cylpoisson_solve_static", "cylpoisson_solve_planes"):
        getattr(L, name).restype = i
        getattr(L, name).argtypes = [vp, vp, vp, d, vp]
    for name in ("cylpoisson_apply", "cylpoisson_dft_forward", "cylpoisson_dft_inverse"):
        getattr(L, name).restype = i
        getattr(L, name).argtypes = [vp, vp, vp, vp]
    L.cylpoisson_plan_get_option.restype = i
    L.cylpoisson_plan_get_option.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(d)]
    L.cylpoisson_autotune.restype = i
    L.cylpoisson_autotune.argtypes = [vp, vp]
    L.cylpoisson_solve_batch.restype = i
    L.cylpoisson_solve_batch.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i,
                                         d, vp, ctypes.POINTER(i)]
    ull, fp = ctypes.c_ulonglong, ctypes.POINTER(ctypes.c_float)
    L.cylpoisson_nn_create.restype = vp
    L.cylpoisson_nn_create.argtypes = [ull]
    L.cylpoisson_nn_destroy.restype = None
    L.cylpoisson_nn_destroy.argtypes = [vp]
    L.cylpoisson_nn_weight_count.restype = i
    L.cylpoisson_nn_weight_count.argtypes = []
    for name in ("cylpoisson_nn_get_weights", "cylpoisson_nn_set_weights", "cylpoisson_nn_get_grads"):
        getattr(L, name).restype = i
        getattr(L, name).argtypes = [vp, fp, i]
    L.cylpoisson_nn_forward.restype = i
    L.cylpoisson_nn_forward.argtypes = [vp, vp, vp, i, i, i, vp]
    L.cylpoisson_nn_loss_grad.restype = i
    L.cylpoisson_nn_loss_grad.argtypes = [vp, vp, vp, i, i, i, ctypes.POINTER(d), vp]
    L.cylpoisson_nn_adam_step.restype = i
    L.cylpoisson_nn_adam_step.argtypes = [vp, ctypes.c_float, vp]
    L.cylpoisson_nn_collect.restype = i
    L.cylpoisson_nn_collect.argtypes = [vp, vp, vp, i, i, ull, vp]
    L.cylpoisson_nn_patch_count.restype = ctypes.c_longlong
    L.cylpoisson_nn_patch_count.argtypes = [vp]
    L.cylpoisson_nn_train.restype = i
    L.cylpoisson_nn_train.argtypes = [vp, i, i, ctypes.c_float, ctypes.POINTER(d), vp]
    L.cylpoisson_plan_set_net.restype = i
    L.cylpoisson_plan_set_net.argtypes = [vp, vp]
    L.cylpoisson_get_stats.restype = i
    L.cylpoisson_get_stats.argtypes = [vp, ctypes.POINTER(Stats)]
    L.cylpoisson_get_info.restype = i
    L.cylpoisson_get_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.cylpoisson_last_error.restype = ctypes.c_char_p
    L.cylpoisson_last_error.argtypes = []
    L.cylpoisson_last_status.restype = i
    L.cylpoisson_last_status.argtypes = []
    L.cylpoisson_status_string.restype = ctypes.c_char_p
    L.cylpoisson_status_string.argtypes = [i]
    _lib = L
    return L


def last_error() -> str:
    return library().cylpoisson_last_error().decode()


def last_status() -> int:
    """``cylpoisson_last_status``: why the last plan creation in this thread failed."""
    return int(library().cylpoisson_last_status())


def status_string(status: int) -> str:
    return library().cylpoisson_status_string(int(status)).decode()


def _ptr(t) -> int:
    if isinstance(t, torch.Tensor):
        if t.dtype != torch.float64:
            raise TypeError("tensors must be torch.float64")
        if not t.is_contiguous():
            raise ValueError("tensors must be contiguous")
        return t.data_ptr()
    return int(t)


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream if torch.cuda.is_available() else 0
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _check(status: int, allow=(OK,)) -> int:
    if status not in allow:
        raise CylPoissonError(status, last_error())
    return status


def plan_create(nr, ntheta, nz, r_in, r_out, dz, bc=(0.0, 0.0, 0.0, 0.0)) -> int:
    """``cylpoisson_plan_create``; returns the plan handle (int) or raises."""
    b = BC(*[float(x) for x in bc])
    h = library().cylpoisson_plan_create(int(nr), int(ntheta), int(nz), float(r_in),
                                         float(r_out), float(dz), ctypes.byref(b))
    if not h:
        raise CylPoissonError(last_status(), last_error())
    return h


def plan_create_mesh(nr, ntheta, nz, r, z, layout=VERTEX, bc=(0.0, 0.0, 0.0, 0.0)) -> int:
    """``cylpoisson_plan_create_mesh``: r and z are sequences of floats (node
    coordinates for VERTEX, the nr - 1 / nz - 1 cell faces for CELL)."""
    need = (nr, nz) if layout == VERTEX else (nr - 1, nz - 1)
    r = [float(x) for x in r]
    z = [float(x) for x in z]
    if (len(r), len(z)) != tuple(need):
        raise ValueError(f"layout {layout} needs {need[0]} radial and {need[1]} axial values, "
                         f"got {len(r)} and {len(z)}")
    b = BC(*[float(x) for x in bc])
    ra = (ctypes.c_double * max(1, len(r)))(*r)
    za = (ctypes.c_double * max(1, len(z)))(*z)
    h = library().cylpoisson_plan_create_mesh(int(nr), int(ntheta), int(nz), ra, za, int(layout),
                                              ctypes.byref(b))
    if not h:
        raise CylPoissonError(last_status(), last_error())
    return h


def plan_destroy(plan) -> None:
    library().cylpoisson_plan_destroy(plan)


def plan_set_option(plan, key: str, value: float) -> None:
    _check(library().cylpoisson_plan_set_option(plan, key.encode(), float(value)))


def plan_get_option(plan, key: str) -> float:
    v = ctypes.c_double()
    _check(library().cylpoisson_plan_get_option(plan, key.encode(), ctypes.byref(v)))
    return v.value


def autotune(plan, stream=None) -> None:
    _check(library().cylpoisson_autotune(plan, _stream(stream)))


def solve_batch(plans, rhos, phis, tol=1e-12, stream=None, allow=(OK,)):
    """``cylpoisson_solve_batch``: returns (batch status, per-problem statuses)."""
    n = len(plans)
    if not (len(rhos) == len(phis) == n):
        raise ValueError("plans, rhos and phis must have the same length")
    arr = ctypes.c_void_p * max(n, 1)
    st = (ctypes.c_int * max(n, 1))()
    status = library().cylpoisson_solve_batch(arr(*[p for p in plans]), arr(*[_ptr(r) for r in rhos]),
                                              arr(*[_ptr(f) for f in phis]), n, float(tol),
                                              _stream(stream), st)
    _check(status, allow)
    return status, [st[i] for i in range(n)]


def solve(plan, rho, phi, tol=1e-12, stream=None, allow=(OK,)) -> int:
    return _check(library().cylpoisson_solve(plan, _ptr(rho), _ptr(phi), float(tol),
                                             _stream(stream)), allow)


def solve_static(plan, rho, phi, tol=1e-12, stream=None, allow=(OK,)) -> int:
    """``cylpoisson_solve_static``: the solve on the library's static device scratch."""
    return _check(library().cylpoisson_solve_static(plan, _ptr(rho), _ptr(phi), float(tol),
                                                    _stream(stream)), allow)


def solve_planes(plan, b, u, tol=1e-12, stream=None, allow=(OK,)) -> int:
    return _check(library().cylpoisson_solve_planes(plan, _ptr(b), _ptr(u), float(tol),
                                                    _stream(stream)), allow)


def apply(plan, phi, rho_out, stream=None) -> None:
    _check(library().cylpoisson_apply(plan, _ptr(phi), _ptr(rho_out), _stream(stream)))


def dft_forward(plan, x, planes, stream=None) -> None:
    _check(library().cylpoisson_dft_forward(plan, _ptr(x), _ptr(planes), _stream(stream)))


def dft_inverse(plan, planes, x, stream=None) -> None:
    _check(library().cylpoisson_dft_inverse(plan, _ptr(planes), _ptr(x), _stream(stream)))


def get_stats(plan) -> dict:
    s = Stats()
    _check(library().cylpoisson_get_stats(plan, ctypes.byref(s)))
    return s.as_dict()


def get_info(plan) -> dict:
    s = Info()
    _check(library().cylpoisson_get_info(plan, ctypes.byref(s)))
    return s.as_dict()


class Plan:
    """A solver plan for one annular grid (see ``cylpoisson_plan_create``)."""

    def __init__(self, nr, ntheta, nz, r_in, r_out, dz, bc=(0.0, 0.0, 0.0, 0.0), **options):
        self.shape = (int(ntheta), int(nz), int(nr))
        self.handle = plan_create(nr, ntheta, nz, r_in, r_out, dz, bc)
        for k, v in options.items():
            plan_set_option(self.handle, k, v)

    @classmethod
    def for_problem(cls, p, **options) -> "Plan":
        return cls(p.nr, p.ntheta, p.nz, p.r_in, p.r_out, p.dz, p.bc, **options)

    @classmethod
    def from_mesh(cls, r, z, ntheta, layout=VERTEX, bc=(0.0, 0.0, 0.0, 0.0), **options) -> "Plan":
        """Plan on an explicit mesh (``cylpoisson_plan_create_mesh``): node
        coordinates for VERTEX, cell faces for CELL (one node per cell centre
        plus the two outer faces)."""
        extra = 0 if layout == VERTEX else 1
        nr, nz = len(r) + extra, len(z) + extra
        self = cls.__new__(cls)
        self.shape = (int(ntheta), int(nz), int(nr))
        self.handle = plan_create_mesh(nr, ntheta, nz, r, z, layout, bc)
        for k, v in options.items():
            plan_set_option(self.handle, k, v)
        return self

    def set_option(self, key, value):
        plan_set_option(self.handle, key, value)

    def get_option(self, key) -> float:
        return plan_get_option(self.handle, key)

    def autotune(self, stream=None) -> None:
        autotune(self.handle, stream)

    def _check_shape(self, *tensors):
        for t in tensors:
            if tuple(t.shape) != self.shape:
                raise ValueError(f"expected a tensor of shape {self.shape}, got {tuple(t.shape)}")

    def solve(self, rho, tol=1e-12, phi=None, stream=None, allow=(OK,)):
        self._check_shape(rho, *(() if phi is None else (phi,)))
        if phi is None:
            phi = torch.empty_like(rho)
        solve(self.handle, rho, phi, tol, stream, allow)
        return phi, get_stats(self.handle)

    def solve_static(self, rho, tol=1e-12, phi=None, stream=None, allow=(OK,)):
        """The same solve on the library's static device scratch (no allocation
        by the library; a phi of None is allocated here by torch)."""
        self._check_shape(rho, *(() if phi is None else (phi,)))
        if phi is None:
            phi = torch.empty_like(rho)
        solve_static(self.handle, rho, phi, tol, stream, allow)
        return phi, get_stats(self.handle)

    def info(self) -> dict:
        return get_info(self.handle)

    def stats(self) -> dict:
        return get_stats(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_plans(plans, rhos, tol=1e-12, stream=None, allow=(OK,)):
    """Batch-solve Plan objects: returns (phis, per-problem stats)."""
    for plan, rho in zip(plans, rhos):
        plan._check_shape(rho)
    phis = [torch.empty_like(r) for r in rhos]
    status, sts = solve_batch([p.handle for p in plans], rhos, phis, tol, stream, allow)
    return phis, [p.stats() for p in plans]


class Net:
    """The learned preconditioner's network (``cylpoisson_nn_*``)."""

    def __init__(self, seed: int = 2024):
        self.handle = library().cylpoisson_nn_create(int(seed))
        if not self.handle:
            raise CylPoissonError(ENOMEM, last_error())

    @staticmethod
    def weight_count() -> int:
        return library().cylpoisson_nn_weight_count()

    def get_weights(self):
        import numpy as np
        out = np.empty(self.weight_count(), dtype=np.float32)
        _check(library().cylpoisson_nn_get_weights(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                   out.size))
        return out

    def set_weights(self, w) -> None:
        import numpy as np
        a = np.ascontiguousarray(w, dtype=np.float32)
        _check(library().cylpoisson_nn_set_weights(self.handle, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                   a.size))

    def get_grads(self):
        import numpy as np
        out = np.empty(self.weight_count(), dtype=np.float32)
        _check(library().cylpoisson_nn_get_grads(self.handle, out.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                                 out.size))
        return out

    @staticmethod
    def _f32(t):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float32 or not t.is_contiguous():
            raise TypeError("network images must be contiguous torch.float32 tensors")
        return t.data_ptr()

    def forward(self, x, stream=None):
        B, H, W, C = x.shape
        if C != 4:
            raise ValueError("the network takes 4 input channels")
        y = torch.empty((B, H, W, 2), dtype=torch.float32, device=x.device)
        _check(library().cylpoisson_nn_forward(self.handle, self._f32(x), self._f32(y), B, H, W, _stream(stream)))
        return y

    def loss_grad(self, x, t, stream=None) -> float:
        B, H, W, _ = x.shape
        loss = ctypes.c_double()
        _check(library().cylpoisson_nn_loss_grad(self.handle, self._f32(x), self._f32(t), B, H, W,
                                                 ctypes.byref(loss), _stream(stream)))
        return loss.value

    def adam_step(self, lr: float, stream=None) -> None:
        _check(library().cylpoisson_nn_adam_step(self.handle, float(lr), _stream(stream)))

    def collect(self, plan, rho, cycles=6, patches_per_cycle=256, seed=1, stream=None) -> None:
        _check(library().cylpoisson_nn_collect(plan.handle, self.handle, _ptr(rho), int(cycles),
                                               int(patches_per_cycle), int(seed), _stream(stream)))

    def patch_count(self) -> int:
        return library().cylpoisson_nn_patch_count(self.handle)

    def train(self, epochs=4, batch=128, lr=1e-3, stream=None) -> float:
        loss = ctypes.c_double()
        _check(library().cylpoisson_nn_train(self.handle, int(epochs), int(batch), float(lr), ctypes.byref(loss),
                                             _stream(stream)))
        return loss.value

    def close(self):
        if getattr(self, "handle", None):
            library().cylpoisson_nn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def plan_set_net(plan, net) -> None:
    _check(library().cylpoisson_plan_set_net(plan.handle, net.handle if net is not None else None))

