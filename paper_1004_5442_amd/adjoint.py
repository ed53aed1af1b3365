"""Gradients of a final-state density through the scheme: hand-written adjoint
kernels behind ``torch.autograd.Function``, with sqrt(N) checkpointing.

Forward:  f^0 = Minv fhat^eq(rho0, u0 = 0, T0);  f^{n+1} = F(f^n; s), n < N;
          rho^N = sum_i f_i^N.
Backward: lam^N = g_rho (every population), then per step, newest first,
          lam^n = (dF/df^n)^T lam^{n+1} and ds += lam^{n+1} . dF/ds
          (``mrt_adjoint_step``), and finally the adjoint of the
          initialisation gives (d/d rho0, d/d T0) (``mrt_init_adjoint``).
The states f^n needed by the backward pass are not all kept: every K-th
state (K ~ sqrt(N)) is stored in the forward pass (``mrt_step_checkpointed``,
which writes it in place), and each segment of K states is recomputed from
its checkpoint (``mrt_adjoint_sweep``; both loops run in the library, the
recomputation of the next segment on a second stream beside the adjoint
steps of the current one), so memory is O(sqrt(N)) states (the checkpoints
and two segments) for one extra forward pass.  Keeping every state instead (segment = 1) measured slower on
the 256^2 / 500-step workload (4.1 x the forward run against 3.3 x): its 500
states stream through HBM, while the sqrt(N) working set stays in the 256 MB
Infinity Cache.  Periodic grids only.
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from .solver import Solver


class DensityMap(torch.autograd.Function):
    """rho^N = Phi(rho0, T0, s) for a periodic grid (u0 = 0)."""

    @staticmethod
    def forward(ctx, rho0: torch.Tensor, T0: torch.Tensor, s: torch.Tensor, solver: Solver,
                gamma: float, dt: float, dx: float, dy: float, nsteps: int,
                segment: Optional[int] = None):
        sv = s.detach().to("cpu", torch.float64)
        solver.ensure_params(gamma, sv.tolist(), dt, dx, dy, 0.0)
        if not any(ctx.needs_input_grad[:3]):
            K = max(1, nsteps)        # no backward to come: one checkpoint, f^0
        else:
            K = int(segment or max(1, math.ceil(math.sqrt(nsteps))))
        dev = rho0.device
        rho0d = rho0.detach().to(dev, torch.float64).contiguous()
        T0d = T0.detach().to(dev, torch.float64).contiguous()
        zero = torch.zeros_like(rho0d)
        a, b = solver.empty_state(), solver.empty_state()
        solver.init_buffer(rho0d, zero, zero, T0d, a)
        checkpoints = [solver.empty_state() for _ in range((nsteps + K - 1) // K)]
        solver.step_checkpointed(a, b, K, nsteps, checkpoints)
        rhoN = torch.empty_like(rho0d)
        solver.density(a, rhoN)
        ctx.solver, ctx.K, ctx.nsteps = solver, K, nsteps
        # the parameters this forward ran with: the solver may be given other
        # ones (another forward, a finite-difference loop) before backward
        ctx.params = (gamma, sv.tolist(), dt, dx, dy)
        ctx.checkpoints = checkpoints
        ctx.save_for_backward(rho0d, T0d)
        ctx.s_meta = (s.device, s.dtype)
        return rhoN

    @staticmethod
    def backward(ctx, g_rhoN: torch.Tensor):
        solver, K, N = ctx.solver, ctx.K, ctx.nsteps
        rho0d, T0d = ctx.saved_tensors
        gamma, s_list, dt, dx, dy = ctx.params
        # only if another forward or a caller changed them since (setting
        # them waits for the stream: the forward's steps would drain before
        # the backward's launches are queued)
        solver.ensure_params(gamma, s_list, dt, dx, dy, 0.0)
        lam, lam2 = solver.empty_state(), solver.empty_state()
        solver.density_adjoint(g_rhoN.detach().to(torch.float64).contiguous(), lam)
        ds = torch.zeros(16, dtype=torch.float64, device=rho0d.device)
        # recomputed states of two segments: the library recomputes the next
        # segment on a second stream while the adjoint steps read the other
        w = max(0, min(K, N) - 1)
        work = [solver.empty_state() for _ in range(2 * w if N > K else w)]
        solver.adjoint_sweep(ctx.checkpoints, K, N, work, lam, lam2, ds)
        del work
        zero = torch.zeros_like(rho0d)
        g_rho, g_T = torch.empty_like(rho0d), torch.empty_like(rho0d)
        solver.init_adjoint(lam, rho0d, zero, zero, T0d, g_rho=g_rho, g_T=g_T)
        sdev, sdt = ctx.s_meta
        ctx.checkpoints = None
        return g_rho, g_T, ds.to(sdev, sdt), None, None, None, None, None, None, None


def density_after(rho0, T0, s, solver: Solver, gamma, dt, dx, dy, nsteps, segment=None):
    """Differentiable rho^N (see DensityMap)."""
    return DensityMap.apply(rho0, T0, s, solver, gamma, dt, dx, dy, nsteps, segment)
