"""Python front end of one grid: a thin wrapper over the C ABI.

PyTorch supplies device memory (the two population buffers are torch
allocations handed to ``mrt_init_grid``) and the stream (the current torch
stream); the scheme itself runs in the library's kernels.
"""
from __future__ import annotations

from ctypes import byref, c_int, c_longlong, c_void_p
from typing import Optional, Sequence

import numpy as np
import torch

from . import lib as L


def _dev_ptr(t: torch.Tensor) -> c_void_p:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    return c_void_p(t.data_ptr())


def _host_ptr(a: np.ndarray) -> c_void_p:
    return c_void_p(a.ctypes.data)


def _param_key(gamma, s, dt, dx, dy, Pr, side_state):
    side = None if side_state is None else tuple(tuple(float(v) for v in st) for st in side_state)
    return (float(gamma), tuple(float(v) for v in s), float(dt), float(dx), float(dy), float(Pr), side)


class Solver:
    """One nx x ny grid of the D2V16 MRT FD-LB scheme on the current GPU."""

    def __init__(self, nx: int, ny: int, precision: str = "fp32_eq64",
                 bc: Sequence[str] = ("periodic",) * 4, stream: Optional[torch.cuda.Stream] = None):
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the MRT solver runs only on the HIP device")
        self.nx, self.ny = int(nx), int(ny)
        self.precision = precision
        self.prec = L.PRECISION[precision]
        self.bc = tuple(bc)
        self.stream = stream or torch.cuda.current_stream()
        nbytes = L.raw().mrt_population_bytes(self.nx, self.ny, self.prec)
        self._bufs = [torch.empty(nbytes, dtype=torch.uint8, device="cuda") for _ in range(2)]
        ptrs = (c_void_p * 2)(self._bufs[0].data_ptr(), self._bufs[1].data_ptr())
        bcs = (c_int * 4)(*[L.BC[b] for b in self.bc])
        h = c_void_p()
        L.check(L.raw().mrt_init_grid(byref(h), self.nx, self.ny, self.prec, bcs, ptrs,
                                      c_void_p(self.stream.cuda_stream)))
        self._h = h
        pitch, plane, origin = c_longlong(), c_longlong(), c_longlong()
        self._check(L.raw().mrt_get_layout(h, byref(pitch), byref(plane), byref(origin)))
        self.pitch, self.plane, self.origin = pitch.value, plane.value, origin.value
        self.params = None
        self.param_key = None       # (gamma, s, dt, dx, dy, Pr, side states) last set

    # ------------------------------------------------------------ plumbing
    def _check(self, rc):
        L.check(rc, self._h)

    @property
    def handle(self):
        return self._h

    @property
    def storage_dtype(self):
        return torch.float64 if self.prec == 0 else torch.float32

    @property
    def cells(self) -> int:
        return self.nx * self.ny

    def population_bytes(self) -> int:
        return L.raw().mrt_population_bytes(self.nx, self.ny, self.prec)

    def empty_state(self) -> torch.Tensor:
        """A device buffer in the library's padded population layout."""
        return torch.zeros(self.population_bytes(), dtype=torch.uint8, device="cuda")

    def buffers(self):
        cur, other = c_void_p(), c_void_p()
        self._check(L.raw().mrt_current_buffer(self._h, byref(cur), byref(other)))
        return cur.value, other.value

    def close(self):
        if getattr(self, "_h", None):
            L.raw().mrt_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- API
    def set_params(self, gamma, s, dt, dx, dy, Pr=0.0, side_state=None):
        p = L.make_params(gamma, s, dt, dx, dy, Pr, side_state)
        self.param_key = None
        self._check(L.raw().mrt_set_params(self._h, byref(p)))
        self.params = p
        self.param_key = _param_key(gamma, s, dt, dx, dy, Pr, side_state)

    def ensure_params(self, gamma, s, dt, dx, dy, Pr=0.0, side_state=None):
        """set_params unless these are the parameters last set (mrt_set_params
        waits for the stream, so repeating it would stall queued work)."""
        if self.param_key != _param_key(gamma, s, dt, dx, dy, Pr, side_state):
            self.set_params(gamma, s, dt, dx, dy, Pr, side_state)

    def set_case(self, case):
        """Parameters and fields from a workloads.Case."""
        self.set_params(case.gamma, case.s, case.dt, case.dx, case.dy, 0.0, case.side_state)
        self.set_fields(case.rho, case.ux, case.uy, case.T)

    def set_fields(self, rho, ux, uy, T):
        if isinstance(rho, torch.Tensor):
            ts = [t.to(device="cuda", dtype=torch.float64).contiguous() for t in (rho, ux, uy, T)]
            self._check(L.raw().mrt_set_fields(self._h, *[_dev_ptr(t) for t in ts], 1))
            self.stream.synchronize()
        else:
            arrs = [np.ascontiguousarray(a, dtype=np.float64).reshape(self.ny, self.nx)
                    for a in (rho, ux, uy, T)]
            self._check(L.raw().mrt_set_fields(self._h, *[_host_ptr(a) for a in arrs], 0))

    def step(self, n: int = 1):
        self._check(L.raw().mrt_step(self._h, int(n)))

    def prepare(self, n: int):
        """Capture the graphs a following step(n) replays (mrt_prepare_steps)."""
        self._check(L.raw().mrt_prepare_steps(self._h, int(n)))

    def sync(self):
        self._check(L.raw().mrt_sync(self._h))

    def moments(self):
        """(rho, ux, uy, T) as host float64 arrays (ny, nx); synchronises."""
        out = [np.empty((self.ny, self.nx)) for _ in range(4)]
        self._check(L.raw().mrt_read_moments(self._h, *[_host_ptr(a) for a in out], 0))
        return tuple(out)

    def moments_device(self):
        out = [torch.empty((self.ny, self.nx), dtype=torch.float64, device="cuda") for _ in range(4)]
        self._check(L.raw().mrt_read_moments(self._h, *[_dev_ptr(t) for t in out], 1))
        return tuple(out)

    def populations(self) -> np.ndarray:
        """Current populations as float64 (16, ny, nx); synchronises."""
        out = np.empty((16, self.ny, self.nx))
        self._check(L.raw().mrt_get_populations(self._h, _host_ptr(out), 0))
        return out

    def set_populations(self, f: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(16, self.ny, self.nx)
        self._check(L.raw().mrt_set_populations(self._h, _host_ptr(f), 0))

    def set_scheme(self, split: bool = False, lw_cross: bool = False):
        """Select a reading of the discretisation (mrt_set_scheme)."""
        flags = (L.SCHEME_SPLIT if split else 0) | (L.SCHEME_LW_CROSS if lw_cross else 0)
        self._check(L.raw().mrt_set_scheme(self._h, flags))

    def set_steps_per_pass(self, steps: int, rows: int = 0):
        """1, 2 or 4 time steps per kernel pass (mrt_set_steps_per_pass);
        rows: band height of the two-step kernel (0: default).  4: the tube
        march, for grids of 1, 2 or 4 periodic rows with fixed-equilibrium x
        sides."""
        self._check(L.raw().mrt_set_steps_per_pass(self._h, int(steps), int(rows)))

    def steps_per_pass(self):
        """(steps per pass, band rows of the kernel that runs)"""
        k, r = c_int(), c_int()
        self._check(L.raw().mrt_get_steps_per_pass(self._h, byref(k), byref(r)))
        return k.value, r.value

    def set_tile(self, rows: int, grid: int = 0):
        self._check(L.raw().mrt_set_tile(self._h, int(rows), int(grid)))

    def tile(self):
        r, g = c_int(), c_int()
        self._check(L.raw().mrt_get_tile(self._h, byref(r), byref(g)))
        return r.value, g.value

    def autotune(self, steps: int = 4):
        self._check(L.raw().mrt_autotune(self._h, int(steps)))
        return self.tile()

    # ------------------------------------------- explicit-buffer operations
    def step_buffers(self, f_in: torch.Tensor, f_out: torch.Tensor):
        self._check(L.raw().mrt_step_buffers(self._h, _dev_ptr(f_in), _dev_ptr(f_out)))

    def step_checkpointed(self, f: torch.Tensor, f_tmp: torch.Tensor, segment: int, nsteps: int,
                          checkpoints: Sequence[torch.Tensor]):
        arr = (c_void_p * max(1, len(checkpoints)))(*[t.data_ptr() for t in checkpoints])
        self._check(L.raw().mrt_step_checkpointed(self._h, _dev_ptr(f), _dev_ptr(f_tmp), int(segment),
                                                  int(nsteps), arr))

    def adjoint_sweep(self, checkpoints: Sequence[torch.Tensor], segment: int, nsteps: int,
                      work: Sequence[torch.Tensor], lam: torch.Tensor, lam_tmp: torch.Tensor,
                      ds: torch.Tensor):
        """work: min(segment, nsteps) - 1 state buffers, or twice as many to
        recompute the next segment on a second stream beside the adjoint
        steps (same results)."""
        ck = (c_void_p * max(1, len(checkpoints)))(*[t.data_ptr() for t in checkpoints])
        wk = (c_void_p * max(1, len(work)))(*[t.data_ptr() for t in work])
        self._check(L.raw().mrt_adjoint_sweep(self._h, ck, int(segment), int(nsteps), wk, len(work),
                                              _dev_ptr(lam), _dev_ptr(lam_tmp), _dev_ptr(ds)))

    def init_buffer(self, rho, ux, uy, T, f: torch.Tensor):
        self._check(L.raw().mrt_init_buffer(self._h, *[_dev_ptr(t) for t in (rho, ux, uy, T)], _dev_ptr(f)))

    def density(self, f: torch.Tensor, out: torch.Tensor):
        self._check(L.raw().mrt_density(self._h, _dev_ptr(f), _dev_ptr(out)))

    def density_adjoint(self, g: torch.Tensor, lam: torch.Tensor):
        self._check(L.raw().mrt_density_adjoint(self._h, _dev_ptr(g), _dev_ptr(lam)))

    def adjoint_step(self, lam_next: torch.Tensor, f_n: torch.Tensor, lam_n: torch.Tensor,
                     ds: torch.Tensor):
        self._check(L.raw().mrt_adjoint_step(self._h, _dev_ptr(lam_next), _dev_ptr(f_n),
                                             _dev_ptr(lam_n), _dev_ptr(ds)))

    def init_adjoint(self, lam0, rho, ux, uy, T, g_rho=None, g_ux=None, g_uy=None, g_T=None):
        nul = c_void_p(None)
        ptr = lambda t: _dev_ptr(t) if t is not None else nul
        self._check(L.raw().mrt_init_adjoint(self._h, _dev_ptr(lam0), *[_dev_ptr(t) for t in (rho, ux, uy, T)],
                                             ptr(g_rho), ptr(g_ux), ptr(g_uy), ptr(g_T)))


def solver_for_case(case, precision: str = "fp32_eq64", stream=None) -> Solver:
    s = Solver(case.nx, case.ny, precision, case.bc, stream)
    s.set_case(case)
    return s
