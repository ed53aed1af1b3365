"""Linear (von Neumann) stability of the scheme about a uniform state.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Linearising one step of ``oracle.mrt.step`` about a uniform state f0 on a
periodic grid, a Fourier mode f' exp(i(k_x x + k_y y)) with phase angles
theta = (k_x dx, k_y dy) is multiplied by
    G(theta) = diag(1 + L_i(theta)) - dt J_C(f0),
where J_C = dC/df (complex step of the oracle collision) and L_i is the
Lax-Wendroff symbol  sum_a [-i c_ia sin(theta_a) + c_ia^2 (cos(theta_a) - 1)].
The paper requires s_5..s_16 in [0, 1/dt] "for linear stability" (text after
Eq. 12d); this tool checks the whole amplification spectrum for a state.
"""
from __future__ import annotations

import numpy as np

from . import mrt
from .adjoint import collision_jacobian


def amplification_matrix(state, p: mrt.Params, theta_x: float, theta_y: float):
    rho, ux, uy, T = state
    f0 = mrt.feq(rho, ux, uy, T, p.b, p.eta0)            # (16,)
    J = collision_jacobian(f0.reshape(mrt.NPOP, 1, 1), p)[:, :, 0, 0]
    cx, cy = mrt.courant_numbers(p)
    cx = cx.ravel()
    cy = cy.ravel()
    sym = (-1j * cx * np.sin(theta_x) + cx * cx * (np.cos(theta_x) - 1.0)
           - 1j * cy * np.sin(theta_y) + cy * cy * (np.cos(theta_y) - 1.0))
    return np.diag(1.0 + sym) - p.dt * J


def max_amplification(state, p: mrt.Params, n_theta: int = 33, one_d: bool = False):
    """max over the theta grid of the spectral radius of G(theta)."""
    thetas = np.linspace(-np.pi, np.pi, n_theta)
    worst = 0.0
    ty_list = [0.0] if one_d else thetas
    for tx in thetas:
        for ty in ty_list:
            G = amplification_matrix(state, p, tx, ty)
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(G)))))
    return worst


def mode_rates(state, p: mrt.Params, theta_x: float, theta_y: float):
    """Eigenvalues of G(theta) sorted by modulus (largest first)."""
    G = amplification_matrix(state, p, theta_x, theta_y)
    ev = np.linalg.eigvals(G)
    return ev[np.argsort(-np.abs(ev))]
