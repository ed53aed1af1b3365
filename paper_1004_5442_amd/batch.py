"""Many independent grids advanced together (the batched form).

All instances share two population buffers; every time step of every
instance is one kernel launch over a table of (instance, tile) work items,
and ``step(n)`` replays a HIP graph of n such launches captured by the
library.  Thin wrapper over the ``mrt_batch_*`` C ABI.
"""
from __future__ import annotations

from ctypes import byref, c_int, c_void_p
from typing import Sequence

import numpy as np
import torch

from . import lib as L


class Batch:
    def __init__(self, cases: Sequence, precision: str = "fp32_eq64", stream=None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the MRT batch runs only on the HIP device")
        self.cases = list(cases)
        self.prec = L.PRECISION[precision]
        self.precision = precision
        self.stream = stream or torch.cuda.current_stream()
        n = len(self.cases)
        descs = (L.Instance * n)()
        for i, c in enumerate(self.cases):
            descs[i].nx, descs[i].ny = c.nx, c.ny
            for k in range(4):
                descs[i].bc[k] = L.BC[c.bc[k]]
            descs[i].params = L.make_params(c.gamma, c.s, c.dt, c.dx, c.dy, 0.0, c.side_state)
        h = c_void_p()
        L.check(L.raw().mrt_batch_create(byref(h), n, descs, self.prec, c_void_p(self.stream.cuda_stream)))
        self._h = h
        for i, c in enumerate(self.cases):
            arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (c.rho, c.ux, c.uy, c.T)]
            self._check(L.raw().mrt_batch_set_fields(h, i, *[c_void_p(a.ctypes.data) for a in arrs]))

    def _check(self, rc):
        L.check(rc, self._h, batch=True)

    @property
    def cells(self) -> int:
        return int(L.raw().mrt_batch_cells(self._h))

    def step(self, n: int = 1):
        self._check(L.raw().mrt_batch_step(self._h, int(n)))

    def prepare(self, n: int):
        """Capture the graphs a following step(n) replays (mrt_batch_prepare_steps)."""
        self._check(L.raw().mrt_batch_prepare_steps(self._h, int(n)))

    def moments(self, i: int):
        c = self.cases[i]
        out = [np.empty((c.ny, c.nx)) for _ in range(4)]
        self._check(L.raw().mrt_batch_read_moments(self._h, i, *[c_void_p(a.ctypes.data) for a in out]))
        return tuple(out)

    def populations(self, i: int) -> np.ndarray:
        c = self.cases[i]
        out = np.empty((16, c.ny, c.nx))
        self._check(L.raw().mrt_batch_get_populations(self._h, i, c_void_p(out.ctypes.data)))
        return out

    def set_tile(self, rows: int, grid: int = 0):
        self._check(L.raw().mrt_batch_set_tile(self._h, int(rows), int(grid)))

    def tile(self):
        r, g = c_int(), c_int()
        self._check(L.raw().mrt_batch_get_tile(self._h, byref(r), byref(g)))
        return r.value, g.value

    def set_steps_per_pass(self, steps: int, rows: int = 0):
        """1, 2 or 4 time steps per kernel pass (mrt_batch_set_steps_per_pass;
        4: the tube march, for batches of tubes of one common height of 1, 2
        or 4 periodic rows with fixed-equilibrium x sides)."""
        self._check(L.raw().mrt_batch_set_steps_per_pass(self._h, int(steps), int(rows)))

    def steps_per_pass(self):
        k, r = c_int(), c_int()
        self._check(L.raw().mrt_batch_get_steps_per_pass(self._h, byref(k), byref(r)))
        return k.value, r.value

    def autotune(self, steps: int = 8):
        self._check(L.raw().mrt_batch_autotune(self._h, int(steps)))
        return self.tile()

    def close(self):
        if getattr(self, "_h", None):
            L.raw().mrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
