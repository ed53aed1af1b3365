"""Discrete adjoint of the oracle's time step and initialisation.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The forward map of one step (Eq. 3 with forward Euler and Lax-Wendroff) is
    F(f)_i(x) = f_i(x) - dt C_i(f(x)) + LW_i(f)(x),
with C the collision of ``oracle.mrt.collision``.  Its adjoint is
    lambda^n = (dF/df^n)^T lambda^{n+1}.
Every derivative here is taken by complex-step differentiation of the
oracle's own forward functions (Im F(x + i h e_k) / h, exact to rounding for
the rational functions of the scheme), so no derivative is worked out by hand.

Periodic boundaries only: with periodic ghosts the Lax-Wendroff map is a
circulant stencil whose transpose is the mirrored stencil.
"""
from __future__ import annotations

import numpy as np

from . import mrt

H = 1e-30   # complex-step size


def _require_periodic(p: mrt.Params):
    if any(k != mrt.BC_PERIODIC for k in p.bc):
        raise ValueError("the oracle adjoint supports periodic boundaries only")


def collision_jacobian(f, p: mrt.Params):
    """J[i, j, ...] = d C_i / d f_j at every cell, by complex step."""
    n = f.shape[0]
    J = np.empty((n, n) + f.shape[1:])
    for j in range(n):
        fc = f.astype(np.complex128)
        fc[j] += 1j * H
        J[:, j] = np.imag(mrt.collision(fc, p)) / H
    return J


def lax_wendroff_transpose(lam, p: mrt.Params):
    """Transpose of the periodic Lax-Wendroff map applied to lam (16, ny, nx).

    Forward, per population and axis: out(x) = a f(x+1) + b f(x) + d f(x-1)
    with a = -c/2 + c^2/2, b = -c^2, d = c/2 + c^2/2.  The transpose sends
    lam(x) to x-1 with weight a, to x with b and to x+1 with d.
    """
    cx, cy = mrt.courant_numbers(p)
    out = np.zeros_like(lam)
    for c, axis in ((cx, 2), (cy, 1)):
        a = -0.5 * c + 0.5 * c * c
        bb = -c * c
        d = 0.5 * c + 0.5 * c * c
        # sum_x lam(x) a f(x+1) = sum_y lam(y-1) a f(y): contribution a*lam(y-1)
        out = out + a * np.roll(lam, 1, axis=axis) + bb * lam + d * np.roll(lam, -1, axis=axis)
    return out


def adjoint_step(lam_next, f_n, p: mrt.Params):
    """lambda^n = (dF/df^n)^T lambda^{n+1} and dL/ds contribution of this step.

    Returns (lam_n, ds) where ds[k] = sum_x sum_i lam_i(x) dF_i(x)/ds_k and
    dF_i/ds_k = -dt Minv_ik (fhat_k - fhat^eq_k): C is linear in s.
    """
    _require_periodic(p)
    J = collision_jacobian(f_n, p)
    lam_n = lam_next + lax_wendroff_transpose(lam_next, p) \
        - p.dt * np.einsum("ij...,i...->j...", J, lam_next)
    M = mrt.transformation_matrix(p.eta0)
    Minv = np.linalg.inv(M)
    m = np.tensordot(M, f_n, axes=(1, 0))
    meq = mrt.equilibrium_moments(m[0], m[1], m[2], m[3], p.b)
    w = np.tensordot(Minv.T, lam_next, axes=(1, 0))      # (Minv^T lam)_k
    ds = -p.dt * np.sum(w * (m - meq), axis=tuple(range(1, f_n.ndim)))
    return lam_n, ds


def init_adjoint(lam0, rho, ux, uy, T, p: mrt.Params):
    """Gradients of <lam0, f^0> w.r.t. the initial fields (rho, ux, uy, T),
    f^0 = Minv fhat^eq(rho, u, T), each by complex step."""
    fields = [np.asarray(a, dtype=np.complex128) for a in (rho, ux, uy, T)]
    grads = []
    for k in range(4):
        args = [a.copy() for a in fields]
        args[k] = args[k] + 1j * H
        df = np.imag(mrt.init_populations(*args, p)) / H
        grads.append(np.sum(lam0 * df, axis=0))
    return grads


def density_misfit_gradient(rho0, ux0, uy0, T0, rho_target, p: mrt.Params, nsteps: int):
    """Loss L = 1/2 sum_x (rho^N - rho_target)^2 and its gradient w.r.t.
    (rho0, ux0, uy0, T0) and s_1..16.

    All forward states are stored (no checkpointing: this is the reference).
    """
    f = mrt.init_populations(rho0, ux0, uy0, T0, p)
    states = [f]
    for _ in range(nsteps):
        f = mrt.step(f, p)
        states.append(f)
    rho_n = np.sum(f, axis=0)                    # fhat_1 = sum_i f_i
    r = rho_n - rho_target
    loss = 0.5 * float(np.sum(r * r))
    lam = np.broadcast_to(r, f.shape).copy()     # dL/df_i = r for every i
    ds = np.zeros(mrt.NPOP)
    for n in range(nsteps - 1, -1, -1):
        lam, ds_n = adjoint_step(lam, states[n], p)
        ds += ds_n
    g_rho, g_ux, g_uy, g_T = init_adjoint(lam, rho0, ux0, uy0, T0, p)
    return loss, {"rho": g_rho, "ux": g_ux, "uy": g_uy, "T": g_T, "s": ds}
