"""Exact solution of the Riemann problem of the 1D Euler equations (ideal gas).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Used to validate the oracle on shock tubes (the paper's section (b) compares
its runs with the exact solution).  Textbook method: the star-region pressure
p* is the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, where f_K is the shock
(Rankine-Hugoniot) branch for p > p_K and the rarefaction (isentropic,
Riemann-invariant) branch for p <= p_K; u* follows from the same functions,
and the solution at x/t is sampled wave by wave (E. F. Toro, "Riemann Solvers
and Numerical Methods for Fluid Dynamics", ch. 4).  Temperature is T = p/rho
(R = 1).
"""
from __future__ import annotations

import math

import numpy as np


def _f_branch(p, rho_k, p_k, gamma):
    """f_K(p) and its derivative."""
    a_k = math.sqrt(gamma * p_k / rho_k)
    if p > p_k:   # shock
        A = 2.0 / ((gamma + 1.0) * rho_k)
        B = (gamma - 1.0) / (gamma + 1.0) * p_k
        q = math.sqrt(A / (p + B))
        return (p - p_k) * q, q * (1.0 - 0.5 * (p - p_k) / (B + p))
    # rarefaction
    e = (gamma - 1.0) / (2.0 * gamma)
    return (2.0 * a_k / (gamma - 1.0)) * ((p / p_k) ** e - 1.0), \
        (1.0 / (rho_k * a_k)) * (p / p_k) ** (-(gamma + 1.0) / (2.0 * gamma))


def star_state(left, right, gamma, tol=1e-14, maxit=200):
    """(p*, u*) for primitive states left/right = (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    al = math.sqrt(gamma * pl / rl)
    ar = math.sqrt(gamma * pr / rr)
    if 2.0 * (al + ar) / (gamma - 1.0) <= ur - ul:
        raise ValueError("vacuum is generated; not handled")
    # two-rarefaction guess, always positive
    e = (gamma - 1.0) / (2.0 * gamma)
    p = ((al + ar - 0.5 * (gamma - 1.0) * (ur - ul))
         / (al / pl ** e + ar / pr ** e)) ** (1.0 / e)
    for _ in range(maxit):
        fl, dl = _f_branch(p, rl, pl, gamma)
        fr, dr = _f_branch(p, rr, pr, gamma)
        p_new = p - (fl + fr + ur - ul) / (dl + dr)
        if p_new <= 0.0:
            p_new = 0.5 * p
        if abs(p_new - p) <= tol * 0.5 * (p_new + p):
            p = p_new
            break
        p = p_new
    fl, _ = _f_branch(p, rl, pl, gamma)
    fr, _ = _f_branch(p, rr, pr, gamma)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def sample(left, right, gamma, xi):
    """(rho, u, p) of the self-similar solution at xi = (x - x0)/t (array)."""
    rl, ul, pl = left
    rr, ur, pr = right
    ps, us = star_state(left, right, gamma)
    g = gamma
    gm = (g - 1.0) / (g + 1.0)
    xi = np.atleast_1d(np.asarray(xi, dtype=float))
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    al = math.sqrt(g * pl / rl)
    ar = math.sqrt(g * pr / rr)
    for n, s in enumerate(xi):
        if s <= us:   # left of the contact
            if ps > pl:   # left shock
                r_star = rl * ((ps / pl) + gm) / (gm * (ps / pl) + 1.0)
                sl = ul - al * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                st = (rl, ul, pl) if s < sl else (r_star, us, ps)
            else:         # left rarefaction
                r_star = rl * (ps / pl) ** (1.0 / g)
                a_star = al * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                head, tail = ul - al, us - a_star
                if s < head:
                    st = (rl, ul, pl)
                elif s > tail:
                    st = (r_star, us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * ul + s)
                    c = 2.0 / (g + 1.0) * (al + 0.5 * (g - 1.0) * (ul - s))
                    rr_ = rl * (c / al) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pl * (c / al) ** (2.0 * g / (g - 1.0)))
        else:         # right of the contact
            if ps > pr:   # right shock
                r_star = rr * ((ps / pr) + gm) / (gm * (ps / pr) + 1.0)
                sr = ur + ar * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                st = (rr, ur, pr) if s > sr else (r_star, us, ps)
            else:         # right rarefaction
                r_star = rr * (ps / pr) ** (1.0 / g)
                a_star = ar * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                head, tail = ur + ar, us + a_star
                if s > head:
                    st = (rr, ur, pr)
                elif s < tail:
                    st = (r_star, us, ps)
                else:
                    uu = 2.0 / (g + 1.0) * (-ar + 0.5 * (g - 1.0) * ur + s)
                    c = 2.0 / (g + 1.0) * (ar - 0.5 * (g - 1.0) * (ur - s))
                    rr_ = rr * (c / ar) ** (2.0 / (g - 1.0))
                    st = (rr_, uu, pr * (c / ar) ** (2.0 * g / (g - 1.0)))
        rho[n], u[n], p[n] = st
    return rho, u, p
