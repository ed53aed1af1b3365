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


# Readings of the paper's discretisation passage ("time evolution ...
# first-order upwind scheme, space discretisation ... Lax-Wendroff", section
# "Construction", last paragraph before Fig. 1) whose linear amplification
# this tool can form.  With L = diag(LW symbol), K = dt J_C:
#   "unsplit"      I + L - K                 forward Euler, collision and
#                                            convection both from f^n (the
#                                            oracle's and the library's)
#   "split"        (I + L)(I - K)            collide, then convect (the oracle's
#                                            ``split`` option); convect-then-
#                                            collide, (I - K)(I + L), has the
#                                            same spectrum
#   "rhs_taylor"   I + L - K - (L1 K + K L1)/2 + K^2/2
#                                            Lax-Wendroff's second-order Taylor
#                                            term applied to the whole right-hand
#                                            side, collision included (L1: the
#                                            first-difference part of L)
#   "trapezoid"    (I + K/2)^-1 (I - K/2)(I + L)
#                                            a Crank-Nicolson collision, then
#                                            convection
#   "exp_collision" exp(-K)(I + L)           the exact linear collision, then
#                                            convection
READINGS = ("unsplit", "split", "rhs_taylor", "trapezoid", "exp_collision")


def _lw_symbols(p: mrt.Params, theta_x: float, theta_y: float):
    cx, cy = mrt.courant_numbers(p)
    cx = cx.ravel()
    cy = cy.ravel()
    first = -1j * cx * np.sin(theta_x) - 1j * cy * np.sin(theta_y)
    second = cx * cx * (np.cos(theta_x) - 1.0) + cy * cy * (np.cos(theta_y) - 1.0)
    return first, second


def amplification_matrix(state, p: mrt.Params, theta_x: float, theta_y: float,
                         reading: str = "unsplit"):
    rho, ux, uy, T = state
    f0 = mrt.feq(rho, ux, uy, T, p.b, p.eta0)            # (16,)
    J = collision_jacobian(f0.reshape(mrt.NPOP, 1, 1), p)[:, :, 0, 0]
    first, second = _lw_symbols(p, theta_x, theta_y)
    eye = np.eye(mrt.NPOP)
    Lmat = np.diag(first + second)
    K = p.dt * J
    if reading == "unsplit":
        return eye + Lmat - K
    if reading == "split":
        return (eye + Lmat) @ (eye - K)
    if reading == "rhs_taylor":
        L1 = np.diag(first)
        return eye + Lmat - K - 0.5 * (L1 @ K + K @ L1) + 0.5 * (K @ K)
    if reading == "trapezoid":
        return np.linalg.solve(eye + 0.5 * K, eye - 0.5 * K) @ (eye + Lmat)
    if reading == "exp_collision":
        w, V = np.linalg.eig(K)
        expK = (V * np.exp(-w)) @ np.linalg.inv(V)
        return expK @ (eye + Lmat)
    raise ValueError(f"unknown reading {reading!r}")


def semi_discrete_growth(state, p: mrt.Params, theta_x: float, theta_y: float = 0.0):
    """Largest real part (per unit time) of the eigenvalues of the model
    continuous in time and space, -i (k . v) - J_C, at the wavenumbers whose
    grid phase angles are (theta_x, theta_y): what remains of a growth rate
    when the time step and the Lax-Wendroff dissipation are taken away."""
    rho, ux, uy, T = state
    f0 = mrt.feq(rho, ux, uy, T, p.b, p.eta0)
    J = collision_jacobian(f0.reshape(mrt.NPOP, 1, 1), p)[:, :, 0, 0]
    vx, vy, _ = mrt.velocity_set(p.eta0)
    A = -1j * np.diag(vx * theta_x / p.dx + vy * theta_y / p.dy) - J
    return float(np.max(np.linalg.eigvals(A).real))


def max_amplification(state, p: mrt.Params, n_theta: int = 33, one_d: bool = False,
                      reading: str = "unsplit"):
    """max over the theta grid of the spectral radius of G(theta)."""
    thetas = np.linspace(-np.pi, np.pi, n_theta)
    worst = 0.0
    ty_list = [0.0] if one_d else thetas
    for tx in thetas:
        for ty in ty_list:
            G = amplification_matrix(state, p, tx, ty, reading)
            worst = max(worst, float(np.max(np.abs(np.linalg.eigvals(G)))))
    return worst


def mode_rates(state, p: mrt.Params, theta_x: float, theta_y: float):
    """Eigenvalues of G(theta) sorted by modulus (largest first)."""
    G = amplification_matrix(state, p, theta_x, theta_y)
    ev = np.linalg.eigvals(G)
    return ev[np.argsort(-np.abs(ev))]
