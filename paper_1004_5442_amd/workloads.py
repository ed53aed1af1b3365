"""Seeded synthetic workloads shaped like the paper's test problems.

This module only builds initial macroscopic fields (rho, ux, uy, T), scheme
parameters and boundary descriptions.  It holds none of the scheme's
arithmetic (no velocity set, no moments, no equilibria, no time step), so
both the HIP path and the independent CPU oracle can take their inputs from
it.  It imports nothing from the rest of the package.

Units: R = 1, so p = rho T and the sound speed is sqrt(gamma T).
Boundary kinds are named by strings: "periodic", "eq" (ghost cells hold the
equilibrium of a fixed state: fixed tube ends, inflow), "outflow"
(zero-gradient copy) and "reflect" (mirror cell with the normal velocity
reversed).  Sides are ordered (x-lo, x-hi, y-lo, y-hi).

Interfaces between initial states are smoothed with a tanh profile of a
stated width in cells where a case says so: with the paper's forward-Euler /
Lax-Wendroff scheme a one-cell jump at a cell Reynolds number far above one
breaks down within a few hundred steps, while a two-cell ramp runs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Sequence, Tuple

import numpy as np

State = Tuple[float, float, float, float]   # (rho, ux, uy, T)


@dataclass
class Case:
    name: str
    nx: int
    ny: int
    rho: np.ndarray
    ux: np.ndarray
    uy: np.ndarray
    T: np.ndarray
    gamma: float
    Pr: float
    s: np.ndarray                       # s_1..s_16 (s[k-1] = s_k), s_8 = s_9 = Pr s_6 already applied
    dt: float
    dx: float
    dy: float
    bc: Tuple[str, str, str, str]
    side_state: Tuple[State, State, State, State]
    nsteps: int
    eta0: float = 2.5
    meta: dict = field(default_factory=dict)

    @property
    def cells(self) -> int:
        return self.nx * self.ny


def rates(s5: float, s6: float, Pr: float, s_rest: float) -> np.ndarray:
    """s_1..4 = 0 (they multiply collision invariants), s_5, s_6 = s_7,
    s_8 = s_9 = Pr s_6, s_10..16 = s_rest."""
    s = np.zeros(16)
    s[4] = s5
    s[5] = s[6] = s6
    s[7] = s[8] = Pr * s6
    s[9:] = s_rest
    return s


def rankine_hugoniot(mach: float, pre: State, gamma: float, direction: int = +1) -> State:
    """State behind a shock of Mach number `mach` running into `pre` (at rest
    in its own frame after removing pre's velocity) in direction +-x."""
    rho1, u1, v1, T1 = pre
    p1 = rho1 * T1
    c1 = np.sqrt(gamma * T1)
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    speed = mach * c1
    u2 = u1 + direction * speed * (1.0 - rho1 / rho2)
    return (float(rho2), float(u2), float(v1), float(p2 / rho2))


def _ramp(d, width_cells, h):
    """0 -> 1 as the signed distance d crosses 0; sharp if width_cells == 0."""
    if width_cells <= 0:
        return (d > 0).astype(float)
    return 0.5 * (1.0 + np.tanh(d / (width_cells * h)))


def _blend(a: State, b: State, w):
    return [a[k] * (1.0 - w) + b[k] * w for k in range(4)]


# ---------------------------------------------------------------------------
# Quasi-1D Sod shock tube (plain method, FP64)
# ---------------------------------------------------------------------------

def sod_tube(nx: int = 400, ny: int = 4, nsteps: int = 1000) -> Case:
    """Sod tube on [0,1] x [0, ny/nx]: left (rho, u, v, p) = (1, 0, 0, 1),
    right (0.125, 0, 0, 0.1), diaphragm on the face x = 0.5, gamma = 1.4,
    Pr = 0.71.  Rates: the paper's 1D Riemann rates (s_5 = 5e3, s_6 = 1e4,
    others 1e5) with s_5 and s_6 divided by 10 (the paper ran at T = 8-77,
    where s_6 = 1e4 gives 8-77x the viscosity it gives on Sod at T ~ 1),
    s_8 = s_9 = Pr s_6, dt = 1e-5.  x ends hold the side equilibria, y is
    periodic."""
    dx = 1.0 / nx
    x = (np.arange(nx) + 0.5) * dx
    left = np.broadcast_to(x < 0.5, (ny, nx))
    L: State = (1.0, 0.0, 0.0, 1.0)
    R: State = (0.125, 0.0, 0.0, 0.8)
    rho = np.where(left, L[0], R[0]).astype(float)
    T = np.where(left, L[3], R[3]).astype(float)
    return Case("sod_400x4_fp64", nx, ny, rho, np.zeros_like(rho), np.zeros_like(rho), T,
                gamma=1.4, Pr=0.71, s=rates(500.0, 1000.0, 0.71, 1e5), dt=1e-5, dx=dx, dy=dx,
                bc=("eq", "eq", "periodic", "periodic"), side_state=(L, R, L, L), nsteps=nsteps)


# ---------------------------------------------------------------------------
# 2D four-quadrant Riemann problem
# ---------------------------------------------------------------------------

def quadrant_states(seed: int, gamma: float = 1.4) -> List[State]:
    """Four states: rho ~ U[0.5,1.5], p ~ U[0.1,1.5], Mach ~ U[0,1.5],
    direction ~ U[0,2pi); quadrants ordered 1 (x>,y>), 2 (x<,y>), 3 (x<,y<),
    4 (x>,y<) as in the paper's section (c)."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.5, 1.5)
        p = rng.uniform(0.1, 1.5)
        T = p / rho
        mach = rng.uniform(0.0, 1.5)
        ang = rng.uniform(0.0, 2.0 * np.pi)
        u = mach * np.sqrt(gamma * T)
        out.append((float(rho), float(u * np.cos(ang)), float(u * np.sin(ang)), float(T)))
    return out


PAPER_QUADRANTS: List[State] = [
    (1.5, 0.0, 0.0, 1.0),
    (0.5323, 1.206, 0.0, 0.3 / 0.5323),
    (0.138, 1.206, 1.206, 0.029 / 0.138),
    (0.5323, 0.0, 1.206, 0.3 / 0.5323),
]


def riemann2d(n: int = 1024, seed: int = 0, nsteps: int = 2000, states=None,
              width_cells: float = 2.0, ny: int = None) -> Case:
    """Four-quadrant Riemann problem on [0,1]^2 (corner at the centre),
    gamma = 1.4, Pr = 1, outflow on all sides.  s_5..s_9 = 5e3 (viscous and
    conductive moments), s_10..16 = 2e5, dt = 5e-6 (s dt = 1 for the fast
    moments).  `ny` < n keeps a centred band of rows (same physics)."""
    st = states if states is not None else quadrant_states(seed)
    h = 1.0 / n
    ny = ny or n
    x = (np.arange(n) + 0.5) * h - 0.5
    y = (np.arange(ny) + 0.5 + (n - ny) // 2) * h - 0.5
    Y, X = np.meshgrid(y, x, indexing="ij")
    wx = _ramp(X, width_cells, h)
    wy = _ramp(Y, width_cells, h)
    weights = [wx * wy, (1 - wx) * wy, (1 - wx) * (1 - wy), wx * (1 - wy)]
    f = [sum(weights[q] * st[q][k] for q in range(4)) for k in range(4)]
    out = st[0]
    return Case(f"riemann2d_{n}x{ny}_seed{seed}", n, ny, f[0], f[1], f[2], f[3],
                gamma=1.4, Pr=1.0, s=rates(5e3, 5e3, 1.0, 2e5), dt=5e-6, dx=h, dy=h,
                bc=("outflow",) * 4, side_state=(out,) * 4, nsteps=nsteps,
                meta={"states": st})


# ---------------------------------------------------------------------------
# Batch of independent shock tubes
# ---------------------------------------------------------------------------

def tube_batch(count: int = 512, seed: int = 0, nsteps: int = 1000,
               nx_range=(200, 4000), ny: int = 4, width_cells: float = 2.0) -> List[Case]:
    """Independent tubes: nx ~ U{200..4000}, dx = 1/nx, gamma ~ U[1.1,1.67],
    Pr ~ U[0.5,2], pressure ratio r ~ logU[2,1000]; left (1, 0, 0, p=1),
    right (rho = r^-0.8, p = 1/r).  dt = 5e-6, s_5 = s_6 = 0.5/dt,
    s_8 = s_9 = Pr s_6, s_10..16 = 1/dt.  x ends hold the side equilibria,
    y periodic, diaphragm ramp of two cells."""
    rng = np.random.default_rng(seed)
    dt = 5e-6
    out = []
    for i in range(count):
        nx = int(rng.integers(nx_range[0], nx_range[1] + 1))
        gamma = float(rng.uniform(1.1, 1.67))
        Pr = float(rng.uniform(0.5, 2.0))
        r = float(np.exp(rng.uniform(np.log(2.0), np.log(1000.0))))
        L: State = (1.0, 0.0, 0.0, 1.0)
        R: State = (r ** -0.8, 0.0, 0.0, r ** -0.2)
        dx = 1.0 / nx
        x = (np.arange(nx) + 0.5) * dx
        w = np.broadcast_to(_ramp(x - 0.5, width_cells, dx), (ny, nx))
        f = _blend(L, R, w)
        out.append(Case(f"tube{i}", nx, ny, *[np.ascontiguousarray(a) for a in f],
                        gamma=gamma, Pr=Pr, s=rates(0.5 / dt, 0.5 / dt, Pr, 1.0 / dt), dt=dt,
                        dx=dx, dy=dx, bc=("eq", "eq", "periodic", "periodic"),
                        side_state=(L, R, L, L), nsteps=nsteps, meta={"pressure_ratio": r}))
    return out


# ---------------------------------------------------------------------------
# Smooth periodic fields for the adjoint
# ---------------------------------------------------------------------------

def smooth_noise(n: int, seed: int, sigma_cells: float = 8.0) -> np.ndarray:
    """Gaussian white noise on an n x n periodic grid, convolved with a
    periodic Gaussian of width sigma_cells (FFT), normalised to unit std."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n))
    k = np.fft.fftfreq(n)
    K2 = k[:, None] ** 2 + k[None, :] ** 2
    out = np.real(np.fft.ifft2(np.fft.fft2(w) * np.exp(-2.0 * np.pi ** 2 * sigma_cells ** 2 * K2)))
    return (out - out.mean()) / out.std()


def adjoint_problem(n: int = 256, seed: int = 0, nsteps: int = 500) -> Tuple[Case, np.ndarray]:
    """Periodic n x n grid, rho0 = 1 + 0.05 n_rho, T0 = 1 + 0.05 n_T, u = 0;
    gamma = 1.4, Pr = 0.71, dt = 1e-4, s_5 = 5e3, s_6 = 1e4, s_8 = Pr s_6,
    s_10..16 = 1e4.  Also returns the target-model temperature T0 + 0.01 n'_T
    (the target density is the forward model run from it)."""
    h = 1.0 / n
    n_rho = smooth_noise(n, 3 * seed + 0)
    n_T = smooth_noise(n, 3 * seed + 1)
    n_T2 = smooth_noise(n, 3 * seed + 2)
    rho = 1.0 + 0.05 * n_rho
    T = 1.0 + 0.05 * n_T
    z = np.zeros_like(rho)
    st: State = (1.0, 0.0, 0.0, 1.0)
    case = Case(f"adjoint_{n}x{n}", n, n, rho, z, z.copy(), T, gamma=1.4, Pr=0.71,
                s=rates(5e3, 1e4, 0.71, 1e4), dt=1e-4, dx=h, dy=h,
                bc=("periodic",) * 4, side_state=(st,) * 4, nsteps=nsteps)
    return case, T + 0.01 * n_T2


# ---------------------------------------------------------------------------
# Large strong-shock run: Mach-5 shock hitting a dense bubble
# ---------------------------------------------------------------------------

def shock_bubble(n: int = 4096, nsteps: int = 5000, T1: float = 0.6, mach: float = 5.0,
                 width_cells: float = 2.0, ny: int = None) -> Case:
    """[0,1]^2, gamma = 1.4, Pr = 0.71.  Pre-shock gas (1, 0, 0, T1); a
    Mach-5 planar shock at x = 0.1 moving +x (post-shock state from the
    Rankine-Hugoniot relations); a bubble of density 3 in pressure
    equilibrium (T = T1/3), centre (0.25, 0.5), radius 0.1.  Reflecting
    walls top and bottom, inflow of the post-shock state on the left,
    outflow on the right.  dt = 5e-6, all rates 2e5 (s dt = 1) except
    s_8 = s_9 = Pr s_6.  `ny` < n keeps a centred band of rows."""
    gamma = 1.4
    h = 1.0 / n
    ny = ny or n
    pre: State = (1.0, 0.0, 0.0, T1)
    post = rankine_hugoniot(mach, pre, gamma, +1)
    bub: State = (3.0, 0.0, 0.0, T1 / 3.0)
    x = (np.arange(n) + 0.5) * h
    y = (np.arange(ny) + 0.5 + (n - ny) // 2) * h
    Y, X = np.meshgrid(y, x, indexing="ij")
    w_shock = _ramp(X - 0.1, width_cells, h)                # 0 behind, 1 ahead
    rr = np.sqrt((X - 0.25) ** 2 + (Y - 0.5) ** 2)
    w_bub = _ramp(0.1 - rr, width_cells, h)                  # 1 inside the bubble
    f = _blend(post, pre, w_shock)
    f = [f[k] * (1 - w_bub) + bub[k] * w_bub for k in range(4)]
    return Case(f"shock_bubble_{n}x{ny}", n, ny, *f, gamma=gamma, Pr=0.71,
                s=rates(2e5, 2e5, 0.71, 2e5), dt=5e-6, dx=h, dy=h,
                bc=("eq", "outflow", "reflect", "reflect"),
                side_state=(post, pre, pre, pre), nsteps=nsteps, meta={"post": post})


# ---------------------------------------------------------------------------
# Richtmyer-Meshkov instability (the paper's section (d))
# ---------------------------------------------------------------------------

RM_STATES = {   # (rho, ux, uy, p) as the paper prints them
    "light": (0.1358, 0.0, 0.0, 1.0),
    "heavy": (1.0, 0.0, 0.0, 1.0),
    "shocked": (3.33333, -2.07063, 0.0, 7.125),
}


def rm_instability(nx: int = 360, ny: int = 100, nsteps: int = 4000, shock_x: float = 0.25,
                   width_cells: float = 2.0) -> Case:
    """Shock-driven Richtmyer-Meshkov instability on [0, 0.36] x [0, 0.1]
    (360 x 100 cells at the paper's size): light gas (rho 0.1358, p 1) left
    of the interface x = 0.24 + 0.005 sin(pi/2 + 40 pi y), heavy gas
    (rho 1, p 1) right of it, and the Mach-2.5 shocked heavy gas
    (3.33333, -2.07063, 0, p = 7.125) right of a planar shock at x = shock_x
    (the paper only says that the shock hits the interface at once; 0.25 is
    five cells right of the interface crests).  gamma = 1.4, dt = 1e-5,
    s_5 = 2e3 and every other rate 1e5 (so Pr = s_8 / s_6 = 1).  Inflow of
    the shocked state on the right, a reflecting wall on the left, periodic
    top and bottom."""
    lx, ly = 0.36, 0.1
    dx, dy = lx / nx, ly / ny
    x = (np.arange(nx) + 0.5) * dx
    y = (np.arange(ny) + 0.5) * dy
    Y, X = np.meshgrid(y, x, indexing="ij")
    prim = {k: (v[0], v[1], v[2], v[3] / v[0]) for k, v in RM_STATES.items()}
    iface = 0.24 + 0.005 * np.sin(np.pi / 2 + 40.0 * np.pi * Y)
    h = min(dx, dy)
    w_heavy = _ramp(X - iface, width_cells, h)             # 0 light, 1 heavy
    w_shock = _ramp(X - shock_x, width_cells, h)           # 1 behind the shock
    f = _blend(prim["light"], prim["heavy"], w_heavy)
    f = _blend(tuple(f), prim["shocked"], w_shock)
    s = np.zeros(16)
    s[4] = 2e3
    s[5:] = 1e5
    shocked = prim["shocked"]
    return Case(f"rm_instability_{nx}x{ny}", nx, ny, *[np.asarray(a, dtype=float) for a in f],
                gamma=1.4, Pr=1.0, s=s, dt=1e-5, dx=dx, dy=dy,
                bc=("reflect", "eq", "periodic", "periodic"),
                side_state=(prim["light"], shocked, shocked, shocked), nsteps=nsteps)


# ---------------------------------------------------------------------------
# The paper's strong-shock Riemann problem (section (b)), MRT and SRT
# ---------------------------------------------------------------------------

STRONG_SHOCK_LEFT: State = (5.99924, 19.5975, 0.0, 76.8254)      # (rho, u1, u2, T)
STRONG_SHOCK_RIGHT: State = (5.99242, -6.19633, 0.0, 7.69222)


def srt_rates(tau: float) -> np.ndarray:
    """Single-relaxation-time (BGK) limit of the MRT collision: every rate
    1/tau (s_1..4 multiply collision invariants and are kept at 0)."""
    s = np.zeros(16)
    s[4:] = 1.0 / tau
    return s


def paper_riemann2d(n: int = 500, srt: bool = False, srt_rate: float = 3e3,
                    width_cells: float = 0.0, nsteps: int = 12000) -> Case:
    """The paper's own two-dimensional Riemann problem (section (c)): the four
    printed quadrant states (PAPER_QUADRANTS; quadrant 1 upper right, counted
    anticlockwise, the corner at the centre), gamma = 1.4 (the printed Mach
    numbers 1.358 and 3.1444 hold for it), dx = dy = 0.002, dt = 1e-5,
    t = 0.12 after 12,000 steps.  MRT: s_8 = s_9 = 2e4, every other rate 3e3
    (so Pr = s_8/s_6 = 6.7).  The paper runs SRT without giving its rate:
    srt_rate sets every rate (default 3e3, the MRT viscous rate).  The paper
    gives no domain: [0, 1]^2 (n = 500) with outflow on every side.  Sharp
    initial interfaces by default (width_cells = 0)."""
    c = riemann2d(n=n, states=PAPER_QUADRANTS, width_cells=width_cells, nsteps=nsteps)
    if srt:
        s = srt_rates(1.0 / srt_rate)
    else:
        s = np.zeros(16)
        s[4:] = 3e3
        s[7] = s[8] = 2e4
    kind = f"srt{srt_rate:g}" if srt else "mrt"
    return Case(f"paper_riemann2d_{kind}_{n}x{n}", n, n, c.rho, c.ux, c.uy, c.T, gamma=1.4,
                Pr=float(s[7] / s[5]), s=s, dt=1e-5, dx=1.0 / n, dy=1.0 / n, bc=c.bc,
                side_state=c.side_state, nsteps=nsteps)


def strong_shock_tube(gamma: float = 1.4, srt: bool = False, nx: int = 1100, ny: int = 1,
                      x0: float = 0.25, nsteps: int = 130000, width_cells: float = 0.0) -> Case:
    """The paper's one-dimensional Riemann problem run with the 2D model:
    left (5.99924, 19.5975, 0, T = 76.8254), right (5.99242, -6.19633, 0,
    T = 7.69222), dx = dy = 0.002, dt = 1e-6, t = 0.13 after 130,000 steps.
    MRT rates s_5 = 5e3, s_6 = 1e4, every other rate 1e5 (so Pr = 10); SRT:
    tau = 1e-5, every rate 1e5.  The paper gives no domain: [0, 2.2] with the
    diaphragm at x0 = 0.25 holds every wave up to t = 0.13 for gamma = 7/5
    and 5/3 with 50 cells to spare at each end, so the fixed-equilibrium ends
    are never reached, as the paper requires.  y is periodic; one row by
    default: with several rows the MRT run carries y-waves that are linearly
    unstable at the hot left state (tests/test_paper_cases.py)."""
    dx = 0.002
    x = (np.arange(nx) + 0.5) * dx
    X = np.broadcast_to(x, (ny, nx))
    w = _ramp(X - x0, width_cells, dx)
    f = _blend(STRONG_SHOCK_LEFT, STRONG_SHOCK_RIGHT, w)
    s = srt_rates(1e-5) if srt else rates(5e3, 1e4, 10.0, 1e5)
    name = f"strong_shock_{'srt' if srt else 'mrt'}_g{gamma:.4f}_{nx}x{ny}"
    return Case(name, nx, ny, *[np.ascontiguousarray(a, dtype=float) for a in f],
                gamma=gamma, Pr=float(s[7] / s[5]), s=s, dt=1e-6, dx=dx, dy=dx,
                bc=("eq", "eq", "periodic", "periodic"),
                side_state=(STRONG_SHOCK_LEFT, STRONG_SHOCK_RIGHT, STRONG_SHOCK_LEFT,
                            STRONG_SHOCK_LEFT), nsteps=nsteps, meta={"x0": x0})
