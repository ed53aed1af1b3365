"""Plain FP64 oracle of the paper's D2V16 MRT finite-difference LB scheme.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Everything here is written from the paper (Chen, Xu, Zhang, Li, Succi, "MRT LB
approach to compressible flows with flexible specific-heat ratio and Prandtl
number", EPL letter) in the order and notation of the paper:

* the discrete velocity set and the extra-dof parameter eta
  (section "Construction of energy-conserving MRT LB model", velocity display);
* the transformation matrix M, rows m_1..m_16 (Appendix);
* the equilibrium kinetic moments fhat^eq_1..16 (Appendix), with
  P = rho R T and e = b rho R T + j^2/rho (definitions under Eqs. 12a-12d),
  gamma = (b+2)/b (same section) and R = 1 (section "Numerical simulation");
* the MRT-LB equation, Eq. (3):
  df_i/dt + v_ia df_i/dx_a = -Minv_il S_lk (fhat_k - fhat^eq_k),
  with the relaxation diagonal in moment space;
* first-order forward time stepping and Lax-Wendroff space differencing
  (section "Construction", last paragraph before Fig. 1);
* f^eq = Minv fhat^eq on boundary nodes (section (b) One-dimensional Riemann
  problem), the reflecting condition (section (d) Richtmyer-Meshkov).

Readings of silent or ambiguous passages (the repository's design notes list
them with reasons):

* velocity order within a shell: axis shells (+x, +y, -x, -y), diagonal
  shells (++, -+, --, +-);
* time advance: unsplit forward Euler, collision and convection both from f^n;
* 2D Lax-Wendroff: the 1D Lax-Wendroff difference applied per axis and summed
  (five-point stencil);
* the two alternative readings of that passage, as options of Params: the
  collide-then-stream split (convection of the post-collision populations,
  ``split``) and the full 2D Lax-Wendroff stencil with the mixed-derivative
  term (nine points, ``lw_cross``);
* grid: cell-centred with one ghost layer per side; "f_i = f_i^eq on the
  boundary nodes" fills the ghost layer;
* reflecting wall: ghost = f^eq(rho, mirrored velocity, T) of the mirror-image
  interior cell (the one adjacent to the ghost);
* outflow (not in the paper): zero-gradient copy of the adjacent interior cell.

Layout: populations are arrays of shape (16, ny, nx); x is the last axis.
All arithmetic is float64 (complex128 when the adjoint module differentiates
by complex step: every function here is written so that it also accepts
complex input).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Sequence

import numpy as np

NPOP = 16

# Boundary kinds, one per side (x-lo, x-hi, y-lo, y-hi).
BC_PERIODIC = 0
BC_EQ = 1        # ghost = f^eq of a fixed state (fixed ends of a tube, inflow)
BC_OUTFLOW = 2   # ghost = copy of the adjacent interior cell
BC_REFLECT = 3   # ghost = f^eq of the mirror-image cell with the normal velocity reversed
BC_NONE = -1     # ghost left as NaN: used only to evaluate the scheme on a window

XLO, XHI, YLO, YHI = 0, 1, 2, 3


# ---------------------------------------------------------------------------
# Velocity model (section "Construction of energy-conserving MRT LB model")
# ---------------------------------------------------------------------------

def velocity_set(eta0: float = 2.5):
    """Return (vx, vy, eta) of the 16-velocity Kataoka-Tsutahara model.

    Shell 1: cyc(+-1, 0); shell 2: cyc(+-6, 0); shell 3: sqrt(2)(+-1, +-1);
    shell 4: (3/sqrt(2))(+-1, +-1).  eta_i = 5/2 on shell 1, 0 elsewhere
    (eta0 is kept as an argument; the paper fixes it to 5/2).
    """
    axis = [(1.0, 0.0), (0.0, 1.0), (-1.0, 0.0), (0.0, -1.0)]
    diag = [(1.0, 1.0), (-1.0, 1.0), (-1.0, -1.0), (1.0, -1.0)]
    r2 = np.sqrt(2.0)
    vel = ([(a, b) for a, b in axis]
           + [(6.0 * a, 6.0 * b) for a, b in axis]
           + [(r2 * a, r2 * b) for a, b in diag]
           + [(3.0 / r2 * a, 3.0 / r2 * b) for a, b in diag])
    vx = np.array([v[0] for v in vel])
    vy = np.array([v[1] for v in vel])
    eta = np.array([eta0] * 4 + [0.0] * 12)
    return vx, vy, eta


def transformation_matrix(eta0: float = 2.5) -> np.ndarray:
    """M with rows m_1..m_16 exactly as listed in the Appendix."""
    vx, vy, eta = velocity_set(eta0)
    v2 = vx * vx + vy * vy
    eps = v2 + eta * eta            # v^2 + eta^2
    dif = vx * vx - vy * vy         # vx^2 - vy^2
    rows = [
        np.ones(NPOP),   # m1  = 1
        vx,              # m2  = vx
        vy,              # m3  = vy
        eps,             # m4  = vx^2 + vy^2 + eta^2
        v2,              # m5  = vx^2 + vy^2
        dif,             # m6  = vx^2 - vy^2
        vx * vy,         # m7  = vx vy
        vx * eps,        # m8  = vx (v^2 + eta^2)
        vy * eps,        # m9  = vy (v^2 + eta^2)
        vx * v2,         # m10 = vx (vx^2 + vy^2)
        vy * v2,         # m11 = vy (vx^2 + vy^2)
        vx * dif,        # m12 = vx (vx^2 - vy^2)
        vy * dif,        # m13 = vy (vx^2 - vy^2)
        v2 * eps,        # m14 = (vx^2 + vy^2)(v^2 + eta^2)
        vx * vy * eps,   # m15 = vx vy (v^2 + eta^2)
        dif * eps,       # m16 = (vx^2 - vy^2)(v^2 + eta^2)
    ]
    return np.array(rows)


def inverse_matrix(eta0: float = 2.5) -> np.ndarray:
    """Minv, f = Minv fhat (Eq. 3 and the text after it).  Library inverse."""
    return np.linalg.inv(transformation_matrix(eta0))


def b_from_gamma(gamma: float) -> float:
    """gamma = (b + 2)/b  =>  b = 2/(gamma - 1)."""
    return 2.0 / (gamma - 1.0)


# ---------------------------------------------------------------------------
# Equilibrium kinetic moments (Appendix)
# ---------------------------------------------------------------------------

def equilibrium_moments(rho, jx, jy, e, b):
    """fhat^eq_1..16 from the conserved moments (Appendix), R = 1.

    P = (e - j^2/rho)/b follows from e = b rho R T + j^2/rho and P = rho R T.
    Returns an array of shape (16,) + shape(rho).
    """
    j2 = jx * jx + jy * jy
    P = (e - j2 / rho) / b
    T = P / rho
    jd = jx * jx - jy * jy
    return np.array([
        rho,                                                        # 1
        jx,                                                         # 2
        jy,                                                         # 3
        e,                                                          # 4
        2.0 * P + j2 / rho,                                         # 5
        jd / rho,                                                   # 6
        jx * jy / rho,                                              # 7
        (e + 2.0 * P) * jx / rho,                                   # 8
        (e + 2.0 * P) * jy / rho,                                   # 9
        (4.0 * P + j2 / rho) * jx / rho,                            # 10
        (4.0 * P + j2 / rho) * jy / rho,                            # 11
        (2.0 * P + jd / rho) * jx / rho,                            # 12
        (-2.0 * P + jd / rho) * jy / rho,                           # 13
        2.0 * (b + 2.0) * rho * T * T + (6.0 + b) * T * j2 / rho
        + j2 * j2 / rho ** 3,                                       # 14
        ((b + 4.0) * P + j2 / rho) * jx * jy / rho ** 2,            # 15
        ((b + 4.0) * P + j2 / rho) * jd / rho ** 2,                 # 16
    ])


def conserved_from_primitive(rho, ux, uy, T, b):
    """(rho, jx, jy, e) with j = rho u and e = b rho T + j^2/rho (R = 1)."""
    jx = rho * ux
    jy = rho * uy
    e = b * rho * T + (jx * jx + jy * jy) / rho
    return rho, jx, jy, e


def feq(rho, ux, uy, T, b, eta0: float = 2.5):
    """Velocity-space equilibrium f^eq = Minv fhat^eq (section (b))."""
    rho = np.asarray(rho)
    mom = equilibrium_moments(*conserved_from_primitive(rho, ux, uy, T, b), b)
    return np.tensordot(inverse_matrix(eta0), mom, axes=(1, 0))


# ---------------------------------------------------------------------------
# Parameters
# ---------------------------------------------------------------------------

@dataclass
class Params:
    """Scheme parameters.  s holds s_1..s_16 (0-based: s[k-1] is s_k)."""
    gamma: float = 1.4
    s: Sequence[float] = field(default_factory=lambda: [0.0] * NPOP)
    dt: float = 1e-5
    dx: float = 1.0
    dy: float = 1.0
    eta0: float = 2.5
    bc: Sequence[int] = (BC_PERIODIC, BC_PERIODIC, BC_PERIODIC, BC_PERIODIC)
    side_state: Sequence[Sequence[float]] = ((1.0, 0.0, 0.0, 1.0),) * 4
    split: bool = False      # collide, then convect the post-collision populations
    lw_cross: bool = False   # add the mixed-derivative term of 2D Lax-Wendroff

    @property
    def b(self) -> float:
        return b_from_gamma(self.gamma)


def rates_with_prandtl(s: Sequence[float], Pr: float) -> np.ndarray:
    """Relaxation rates with s_8 = s_9 = Pr * s_6.

    Eqs. (12b)-(12d) give the shear viscosity rho R T / s_6 (= rho R T / s_7)
    and the heat conductivity (b/2 + 1) R rho R T / s_8 (isotropy: s_8 = s_9),
    so Pr = c_p mu / kappa = s_8 / s_6.
    """
    out = np.array(s, dtype=float).copy()
    out[7] = Pr * out[5]
    out[8] = Pr * out[5]
    return out


# ---------------------------------------------------------------------------
# Macroscopic moments
# ---------------------------------------------------------------------------

def kinetic_moments(f, eta0: float = 2.5):
    """fhat = M f for every cell; f has shape (16, ...)."""
    return np.tensordot(transformation_matrix(eta0), f, axes=(1, 0))


def macroscopic(f, b, eta0: float = 2.5):
    """(rho, ux, uy, T) from fhat_1..4 = (rho, jx, jy, e), R = 1."""
    m = kinetic_moments(f, eta0)
    rho, jx, jy, e = m[0], m[1], m[2], m[3]
    ux = jx / rho
    uy = jy / rho
    T = (e - (jx * jx + jy * jy) / rho) / (b * rho)
    return rho, ux, uy, T


def init_populations(rho, ux, uy, T, p: Params):
    """Initial populations f = Minv fhat^eq(rho, u, T) on every cell."""
    return feq(np.asarray(rho), np.asarray(ux), np.asarray(uy), np.asarray(T), p.b, p.eta0)


# ---------------------------------------------------------------------------
# Collision (Eq. 3, right-hand side)
# ---------------------------------------------------------------------------

def collision(f, p: Params):
    """C = Minv diag(s) (M f - fhat^eq(rho, j, e)): the term that Eq. (3)
    subtracts from df/dt.  f has shape (16, ...)."""
    M = transformation_matrix(p.eta0)
    Minv = np.linalg.inv(M)
    m = np.tensordot(M, f, axes=(1, 0))
    meq = equilibrium_moments(m[0], m[1], m[2], m[3], p.b)
    s = np.asarray(p.s, dtype=float).reshape((NPOP,) + (1,) * (f.ndim - 1))
    return np.tensordot(Minv, s * (m - meq), axes=(1, 0))


# ---------------------------------------------------------------------------
# Ghost layer
# ---------------------------------------------------------------------------

def _reflected_eq(f_cells, normal_axis: str, p: Params):
    """f^eq of cells with the velocity component along normal_axis reversed."""
    rho, ux, uy, T = macroscopic(f_cells, p.b, p.eta0)
    if normal_axis == "x":
        ux = -ux
    else:
        uy = -uy
    return feq(rho, ux, uy, T, p.b, p.eta0)


def fill_ghosts(f, p: Params):
    """Return f padded with one ghost layer, shape (16, ny+2, nx+2).

    The x sides are filled first (rows 1..ny); the y sides are then filled
    over the whole padded width, so a corner ghost is the y side's rule
    applied to the x-side ghost next to it.  Only the nine-point stencil
    (lw_cross) reads corners.
    """
    n, ny, nx = f.shape
    g = np.full((n, ny + 2, nx + 2), np.nan, dtype=np.result_type(f.dtype, np.float64))
    g[:, 1:-1, 1:-1] = f
    bc = list(p.bc)
    if (bc[XLO] == BC_PERIODIC) != (bc[XHI] == BC_PERIODIC):
        raise ValueError("periodic x needs both x sides periodic")
    if (bc[YLO] == BC_PERIODIC) != (bc[YHI] == BC_PERIODIC):
        raise ValueError("periodic y needs both y sides periodic")

    # x sides: ghost columns 0 and nx+1, rows 1..ny
    for side, gcol, icol, wcol in ((XLO, 0, 0, nx - 1), (XHI, nx + 1, nx - 1, 0)):
        kind = bc[side]
        if kind == BC_PERIODIC:
            g[:, 1:-1, gcol] = f[:, :, wcol]
        elif kind == BC_EQ:
            r, u, v, t = p.side_state[side]
            g[:, 1:-1, gcol] = feq(r, u, v, t, p.b, p.eta0)[:, None]
        elif kind == BC_OUTFLOW:
            g[:, 1:-1, gcol] = f[:, :, icol]
        elif kind == BC_REFLECT:
            g[:, 1:-1, gcol] = _reflected_eq(f[:, :, icol], "x", p)
        elif kind == BC_NONE:
            pass
        else:
            raise ValueError(f"unknown boundary kind {kind}")

    # y sides: ghost rows 0 and ny+1, all nx+2 columns (padded rows irow + 1
    # and wrow + 1 already hold their x ghosts)
    for side, grow, irow, wrow in ((YLO, 0, 0, ny - 1), (YHI, ny + 1, ny - 1, 0)):
        kind = bc[side]
        if kind == BC_PERIODIC:
            g[:, grow, :] = g[:, wrow + 1, :]
        elif kind == BC_EQ:
            r, u, v, t = p.side_state[side]
            g[:, grow, :] = feq(r, u, v, t, p.b, p.eta0)[:, None]
        elif kind == BC_OUTFLOW:
            g[:, grow, :] = g[:, irow + 1, :]
        elif kind == BC_REFLECT:
            g[:, grow, :] = _reflected_eq(g[:, irow + 1, :], "y", p)
        elif kind == BC_NONE:
            pass
        else:
            raise ValueError(f"unknown boundary kind {kind}")
    return g


# ---------------------------------------------------------------------------
# Convection: Lax-Wendroff per axis
# ---------------------------------------------------------------------------

def courant_numbers(p: Params):
    """c_ia = v_ia dt / dx_a, shape (16, 1, 1) each."""
    vx, vy, _ = velocity_set(p.eta0)
    cx = (vx * p.dt / p.dx).reshape(NPOP, 1, 1)
    cy = (vy * p.dt / p.dy).reshape(NPOP, 1, 1)
    return cx, cy


def lax_wendroff(g, p: Params):
    """Lax-Wendroff increment of -dt v . grad f from the padded array g.

    For one axis with Courant number c the 1D Lax-Wendroff update of
    df/dt + v df/dx = 0 is
        -c/2 (f[x+1] - f[x-1]) + c^2/2 (f[x+1] - 2 f[x] + f[x-1]);
    the two axes are summed.  With p.lw_cross the second-order Taylor term
    dt^2 v_x v_y d2f/dxdy of the 2D scheme is added, with the central
    difference d2f/dxdy = (f[x+1,y+1] - f[x-1,y+1] - f[x+1,y-1] + f[x-1,y-1])
    / (4 dx dy): the increment (c_x c_y / 4) (NE - NW - SE + SW).
    """
    cx, cy = courant_numbers(p)
    c = g[:, 1:-1, 1:-1]
    east = g[:, 1:-1, 2:]
    west = g[:, 1:-1, :-2]
    north = g[:, 2:, 1:-1]
    south = g[:, :-2, 1:-1]
    out = (-0.5 * cx * (east - west) + 0.5 * cx * cx * (east - 2.0 * c + west)
           - 0.5 * cy * (north - south) + 0.5 * cy * cy * (north - 2.0 * c + south))
    if p.lw_cross:
        ne, nw = g[:, 2:, 2:], g[:, 2:, :-2]
        se, sw = g[:, :-2, 2:], g[:, :-2, :-2]
        out = out + 0.25 * cx * cy * (ne - nw - se + sw)
    return out


# ---------------------------------------------------------------------------
# Time step
# ---------------------------------------------------------------------------

def step(f, p: Params):
    """One time step: f^{n+1} = f^n - dt C(f^n) + LW(f^n) (forward Euler).

    With p.split the populations collide first and the post-collision
    populations h = f - dt C(f) are convected: f^{n+1} = h + LW(h).  The
    collision acts on the ghost cells too, which leaves them what the
    boundary rules give for h (an equilibrium ghost does not change under
    collision, and a copied ghost collides like its source cell).
    """
    g = fill_ghosts(f, p)
    if p.split:
        h = g - p.dt * collision(g, p)
        return h[:, 1:-1, 1:-1] + lax_wendroff(h, p)
    return f - p.dt * collision(f, p) + lax_wendroff(g, p)


def run(f, p: Params, nsteps: int):
    for _ in range(nsteps):
        f = step(f, p)
    return f


# ---------------------------------------------------------------------------
# Evaluation on a window of a large grid
# ---------------------------------------------------------------------------

def evolve_window(rho, ux, uy, T, p: Params, x0: int, x1: int, y0: int, y1: int,
                  nsteps: int):
    """Evolve the cells [y0, y1) x [x0, x1) of a large grid for nsteps steps.

    The window starts from the initial equilibrium of the given global fields
    (shape (ny, nx)).  Sides of the window that are domain sides keep their
    boundary condition; sides inside the domain get BC_NONE (NaN ghosts), so
    that every cell whose result depends on data outside the window comes
    out NaN.  Periodic directions must be covered in full.
    Returns the window populations after nsteps (NaN where unknown).
    """
    ny, nx = np.shape(rho)
    x0, x1 = max(0, x0), min(nx, x1)
    y0, y1 = max(0, y0), min(ny, y1)
    bc = list(p.bc)
    if bc[XLO] == BC_PERIODIC and not (x0 == 0 and x1 == nx):
        raise ValueError("window must span the full periodic x extent")
    if bc[YLO] == BC_PERIODIC and not (y0 == 0 and y1 == ny):
        raise ValueError("window must span the full periodic y extent")
    wbc = [bc[XLO] if x0 == 0 else BC_NONE, bc[XHI] if x1 == nx else BC_NONE,
           bc[YLO] if y0 == 0 else BC_NONE, bc[YHI] if y1 == ny else BC_NONE]
    wp = Params(gamma=p.gamma, s=p.s, dt=p.dt, dx=p.dx, dy=p.dy, eta0=p.eta0,
                bc=wbc, side_state=p.side_state, split=p.split, lw_cross=p.lw_cross)
    sl = (slice(y0, y1), slice(x0, x1))
    f = init_populations(np.asarray(rho)[sl], np.asarray(ux)[sl],
                         np.asarray(uy)[sl], np.asarray(T)[sl], wp)
    for _ in range(nsteps):
        f = step(f, wp)
    return f, (x0, x1, y0, y1)
