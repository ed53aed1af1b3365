"""ctypes binding of libmrtlb.so (the C ABI in include/mrtlb.h).

Argument marshalling only: every step of the scheme runs in the library's
HIP kernels.  The library must have been built (``__graft_entry__.build()``
or ``python -m paper_1004_5442_amd.build_lib``); importing this module
without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int, c_longlong, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; MRTLB_LIBRARY names another build of the same sources
# (the host-sanitizer test loads one built with address/undefined checks)
LIB_PATH = os.environ.get("MRTLB_LIBRARY") or os.path.join(HERE, "libmrtlb.so")

MRT_OK, MRT_EINVAL, MRT_EDEVICE, MRT_ESTATE, MRT_EUNSTABLE, MRT_ENOMEM = 0, -1, -2, -3, -4, -5
PRECISION = {"fp64": 0, "fp32": 1, "fp32_eq64": 2}
BC = {"periodic": 0, "eq": 1, "outflow": 2, "reflect": 3}
SCHEME_SPLIT, SCHEME_LW_CROSS = 1, 2
STATUS = {0: "MRT_OK", -1: "MRT_EINVAL", -2: "MRT_EDEVICE", -3: "MRT_ESTATE",
          -4: "MRT_EUNSTABLE", -5: "MRT_ENOMEM"}


class Params(ctypes.Structure):
    _fields_ = [("gamma", c_double), ("Pr", c_double), ("s", c_double * 16),
                ("dt", c_double), ("dx", c_double), ("dy", c_double), ("eta0", c_double),
                ("side_state", (c_double * 4) * 4)]


class Instance(ctypes.Structure):
    _fields_ = [("nx", c_int), ("ny", c_int), ("bc", c_int * 4), ("params", Params)]


class MRTError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class UnstableError(MRTError):
    pass


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

_D = POINTER(c_double)
_F = POINTER(c_float)
_proto = {
    "mrt_init_grid": (c_int, [POINTER(c_void_p), c_int, c_int, c_int, POINTER(c_int), POINTER(c_void_p), c_void_p]),
    "mrt_population_bytes": (c_longlong, [c_int, c_int, c_int]),
    "mrt_get_layout": (c_int, [c_void_p, POINTER(c_longlong), POINTER(c_longlong), POINTER(c_longlong)]),
    "mrt_set_params": (c_int, [c_void_p, POINTER(Params)]),
    "mrt_set_fields": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "mrt_step": (c_int, [c_void_p, c_int]),
    "mrt_prepare_steps": (c_int, [c_void_p, c_int]),
    "mrt_read_moments": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_int]),
    "mrt_get_populations": (c_int, [c_void_p, c_void_p, c_int]),
    "mrt_set_populations": (c_int, [c_void_p, c_void_p, c_int]),
    "mrt_current_buffer": (c_int, [c_void_p, POINTER(c_void_p), POINTER(c_void_p)]),
    "mrt_sync": (c_int, [c_void_p]),
    "mrt_set_tile": (c_int, [c_void_p, c_int, c_int]),
    "mrt_get_tile": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "mrt_set_scheme": (c_int, [c_void_p, c_int]),
    "mrt_set_steps_per_pass": (c_int, [c_void_p, c_int, c_int]),
    "mrt_get_steps_per_pass": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "mrt_autotune": (c_int, [c_void_p, c_int]),
    "mrt_destroy": (None, [c_void_p]),
    "mrt_last_error": (ctypes.c_char_p, [c_void_p]),
    "mrt_adjoint_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mrt_adjoint_step_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mrt_step_buffers": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mrt_step_checkpointed": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, POINTER(c_void_p)]),
    "mrt_adjoint_sweep": (c_int, [c_void_p, POINTER(c_void_p), c_int, c_int, POINTER(c_void_p),
                                  c_int, c_void_p, c_void_p, c_void_p]),
    "mrt_density": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mrt_density_adjoint": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mrt_init_adjoint": (c_int, [c_void_p] + [c_void_p] * 9),
    "mrt_init_buffer": (c_int, [c_void_p] + [c_void_p] * 5),
    "mrt_batch_create": (c_int, [POINTER(c_void_p), c_int, POINTER(Instance), c_int, c_void_p]),
    "mrt_batch_set_fields": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mrt_batch_step": (c_int, [c_void_p, c_int]),
    "mrt_batch_prepare_steps": (c_int, [c_void_p, c_int]),
    "mrt_batch_read_moments": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mrt_batch_get_populations": (c_int, [c_void_p, c_int, c_void_p]),
    "mrt_batch_set_tile": (c_int, [c_void_p, c_int, c_int]),
    "mrt_batch_get_tile": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "mrt_batch_set_steps_per_pass": (c_int, [c_void_p, c_int, c_int]),
    "mrt_batch_get_steps_per_pass": (c_int, [c_void_p, POINTER(c_int), POINTER(c_int)]),
    "mrt_batch_autotune": (c_int, [c_void_p, c_int]),
    "mrt_batch_cells": (c_longlong, [c_void_p]),
    "mrt_batch_destroy": (None, [c_void_p]),
    "mrt_batch_last_error": (ctypes.c_char_p, [c_void_p]),
    "mrt_host_transform": (c_int, [c_int, _D, _D]),
    "mrt_host_equilibrium": (c_int, [c_double, c_double, c_double, c_double, c_double, _D]),
    "mrt_host_collision": (c_int, [c_double, _D, c_double, _D, _D]),
    "mrt_host_cell_adjoint": (c_int, [c_double, _D, c_double, _D, _D, _D, _D]),
    "mrt_host_conserved_fp32": (c_int, [_F, _F]),
}
for _name, (_res, _args) in _proto.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

EXPORTED = tuple(_proto)


def raw():
    """The loaded ctypes library."""
    return _lib


def check(rc: int, handle=None, batch: bool = False):
    if rc == MRT_OK:
        return
    msg = ""
    if handle is not None:
        fn = _lib.mrt_batch_last_error if batch else _lib.mrt_last_error
        m = fn(handle)
        msg = m.decode() if m else ""
    cls = UnstableError if rc == MRT_EUNSTABLE else MRTError
    raise cls(rc, msg)


def make_params(gamma, s, dt, dx, dy, Pr=0.0, side_state=None, eta0=2.5) -> Params:
    p = Params()
    p.gamma = float(gamma)
    p.Pr = float(Pr)
    for k in range(16):
        p.s[k] = float(s[k])
    p.dt, p.dx, p.dy, p.eta0 = float(dt), float(dx), float(dy), float(eta0)
    st = side_state if side_state is not None else [(1.0, 0.0, 0.0, 1.0)] * 4
    for i in range(4):
        for j in range(4):
            p.side_state[i][j] = float(st[i][j])
    return p


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def host_transform(which: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty(16)
    check(_lib.mrt_host_transform(which, _dptr(x), _dptr(out)))
    return out


def host_equilibrium(gamma, rho, ux, uy, T) -> np.ndarray:
    out = np.empty(16)
    check(_lib.mrt_host_equilibrium(gamma, rho, ux, uy, T, _dptr(out)))
    return out


def host_collision(gamma, s, dt, f) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty(16)
    check(_lib.mrt_host_collision(gamma, _dptr(s), dt, _dptr(f), _dptr(out)))
    return out


def host_cell_adjoint(gamma, s, dt, f, lam):
    s = np.ascontiguousarray(s, dtype=np.float64)
    f = np.ascontiguousarray(f, dtype=np.float64)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    coll, dsk = np.empty(16), np.empty(16)
    check(_lib.mrt_host_cell_adjoint(gamma, _dptr(s), dt, _dptr(f), _dptr(lam), _dptr(coll), _dptr(dsk)))
    return coll, dsk


def host_conserved_fp32(f):
    """(rho, jx, jy, e) of 16 FP32 populations as the all-FP32 form computes
    them (compensated FP32 sums)."""
    f = np.ascontiguousarray(f, dtype=np.float32)
    q = np.empty(4, dtype=np.float32)
    check(_lib.mrt_host_conserved_fp32(f.ctypes.data_as(_F), q.ctypes.data_as(_F)))
    return q
