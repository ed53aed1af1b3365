"""Shared test helpers: map seeded workloads onto the oracle, compare fields."""
import numpy as np

from oracle import mrt

BCMAP = {"periodic": mrt.BC_PERIODIC, "eq": mrt.BC_EQ, "outflow": mrt.BC_OUTFLOW,
         "reflect": mrt.BC_REFLECT}


def oracle_params(case, split=False, lw_cross=False):
    return mrt.Params(gamma=case.gamma, s=case.s, dt=case.dt, dx=case.dx, dy=case.dy,
                      eta0=case.eta0, bc=[BCMAP[b] for b in case.bc], side_state=case.side_state,
                      split=split, lw_cross=lw_cross)


def oracle_run(case, nsteps, split=False, lw_cross=False):
    p = oracle_params(case, split, lw_cross)
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


def fp32_storage_reference(case, nsteps):
    """The oracle with every population rounded to float32 after each step:
    what storing f in FP32 alone costs (no other change to the arithmetic)."""
    p = oracle_params(case)
    f = mrt.init_populations(case.rho, case.ux, case.uy, case.T, p)
    f = f.astype(np.float32).astype(np.float64)
    for _ in range(nsteps):
        f = mrt.step(f, p).astype(np.float32).astype(np.float64)
    return f, p


def fp32_tolerances(case, nsteps, want64, floor=1e-5):
    """Per-field tolerance of an FP32-storage run against the FP64 oracle:
    the stated 1e-5, or twice the error that FP32 storage alone produces on
    this workload when that is larger (strong shocks, low densities)."""
    f32, p = fp32_storage_reference(case, nsteps)
    base = field_errors(mrt.macroscopic(f32, p.b), mrt.macroscopic(want64, p.b))
    return {k: max(floor, 2.0 * v) for k, v in base.items()}


def fp64_rounding_spread(case, nsteps, want, seed=0):
    """How far one-ulp rounding differences move an FP64 run: the oracle
    rerun with every population multiplied by (1 +- 2^-52) (random sign)
    after each step, compared with the plain oracle result `want` (relative
    to the population scale).  Two correct FP64 implementations that order
    or fuse their operations differently differ by about this much; on
    well-conditioned cases it is ~1e-14, on the paper's hot supersonic
    strong-shock states (populations far larger than the density they sum
    to) ~1e-10 after 2000 steps."""
    p = oracle_params(case)
    rng = np.random.default_rng(seed)
    f = mrt.init_populations(case.rho, case.ux, case.uy, case.T, p)
    for _ in range(nsteps):
        f = mrt.step(f, p)
        f = f * (1.0 + np.ldexp(rng.choice([-1.0, 1.0], size=f.shape), -52))
    return float(np.max(np.abs(f - want)) / np.abs(want).max())


def one_row(case):
    """The same case on a single periodic row: for a case that is uniform in
    y with periodic y sides (the shock tubes) every row of the oracle does
    the same arithmetic on the same values, and the y increments of a
    uniform column are exactly zero, so the one-row oracle run gives the
    rows of the full one bit for bit at a fraction of the cost (checked by
    tests/test_workloads.py)."""
    import dataclasses
    assert case.bc[2] == case.bc[3] == "periodic"
    for a in (case.rho, case.ux, case.uy, case.T):
        assert np.all(a == a[:1]), "the case is not uniform in y"
    return dataclasses.replace(case, ny=1, rho=case.rho[:1].copy(), ux=case.ux[:1].copy(),
                               uy=case.uy[:1].copy(), T=case.T[:1].copy())
