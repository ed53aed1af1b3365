"""Shared test helpers: map seeded workloads onto the oracle, compare fields."""
import numpy as np

from oracle import mrt

BCMAP = {"periodic": mrt.BC_PERIODIC, "eq": mrt.BC_EQ, "outflow": mrt.BC_OUTFLOW,
         "reflect": mrt.BC_REFLECT}


def oracle_params(case):
    return mrt.Params(gamma=case.gamma, s=case.s, dt=case.dt, dx=case.dx, dy=case.dy,
                      eta0=case.eta0, bc=[BCMAP[b] for b in case.bc], side_state=case.side_state)


def oracle_run(case, nsteps):
    p = oracle_params(case)
    f = mrt.init_populations(case.rho, case.ux, case.uy, case.T, p)
    return mrt.run(f, p, nsteps), p


def field_errors(got, want):
    """Normwise relative error per field: max|a-b| / max|b| for rho and T,
    and max|u - u_ref| / max(|u_ref|, sound speed) for the velocity."""
    r1, u1, v1, T1 = got
    r0, u0, v0, T0 = want
    cs = np.sqrt(np.max(T0))
    sp = max(np.max(np.hypot(u0, v0)), cs)
    return {
        "rho": float(np.max(np.abs(r1 - r0)) / np.max(np.abs(r0))),
        "u": float(max(np.max(np.abs(u1 - u0)), np.max(np.abs(v1 - v0))) / sp),
        "T": float(np.max(np.abs(T1 - T0)) / np.max(np.abs(T0))),
    }


def smooth_case(nx, ny, bc, seed=0, gamma=1.4, amp=0.1, dt=2e-5, side=None):
    """Smooth random fields (a few Fourier modes) for parity on small grids."""
    from paper_1004_5442_amd import workloads as W
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx, indexing="ij")

    def field():
        out = np.zeros((ny, nx))
        for _ in range(4):
            kx, ky = rng.integers(1, 4, 2)
            out += rng.standard_normal() * np.cos(2 * np.pi * (kx * x + ky * y) + rng.uniform(0, 6.3))
        return out / 4

    rho = 1 + amp * field()
    T = 1 + amp * field()
    ux = 2 * amp * field()
    uy = 2 * amp * field()
    h = 1.0 / max(nx, ny)
    st = side or ((1.1, 0.1, 0.0, 0.9), (0.9, -0.1, 0.05, 1.1), (1.0, 0.0, 0.1, 1.0), (1.05, 0.0, -0.1, 1.0))
    return W.Case(f"smooth_{nx}x{ny}", nx, ny, rho, ux, uy, T, gamma=gamma, Pr=0.71,
                  s=W.rates(2e4, 3e4, 0.71, 5e4), dt=dt, dx=h, dy=h, bc=tuple(bc),
                  side_state=st, nsteps=0)
