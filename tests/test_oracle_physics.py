"""Pins of the oracle's time step: conservation, free streaming, boundaries,
and the physics the paper validates against (sound speed, exact Riemann
solution, transport coefficients of Eqs. 12a-12d).
"""
import numpy as np
import pytest

from oracle import mrt, riemann, stability

RNG = np.random.default_rng(7)


def rates(s5, s6, s8, rest):
    s = np.zeros(16)
    s[4] = s5
    s[5] = s[6] = s6
    s[7] = s[8] = s8
    s[9:] = rest
    return s


def test_uniform_state_stays_uniform_all_boundaries():
    st = (0.8, 0.3, -0.2, 1.3)
    p = mrt.Params(gamma=1.4, s=rates(500, 1000, 710, 1e4), dt=2e-5, dx=0.01, dy=0.02,
                   bc=(mrt.BC_EQ, mrt.BC_OUTFLOW, mrt.BC_PERIODIC, mrt.BC_PERIODIC),
                   side_state=(st,) * 4)
    f0 = mrt.feq(*[np.full((5, 7), v) for v in st], p.b)
    f = mrt.run(f0, p, 20)
    np.testing.assert_allclose(f, f0, rtol=0, atol=1e-14)
    # reflecting walls keep a state with no normal velocity
    st2 = (1.1, 0.4, 0.0, 0.9)
    p2 = mrt.Params(gamma=5 / 3, s=rates(500, 1000, 710, 1e4), dt=2e-5, dx=0.01, dy=0.01,
                    bc=(mrt.BC_PERIODIC, mrt.BC_PERIODIC, mrt.BC_REFLECT, mrt.BC_REFLECT))
    f0 = mrt.feq(*[np.full((6, 4), v) for v in st2], p2.b)
    np.testing.assert_allclose(mrt.run(f0, p2, 20), f0, rtol=0, atol=1e-14)


def _smooth_field(ny, nx, amp):
    y, x = np.meshgrid(np.arange(ny) / ny, np.arange(nx) / nx, indexing="ij")
    return amp * (np.sin(2 * np.pi * x + 0.3) * np.cos(4 * np.pi * y) + 0.5 * np.cos(2 * np.pi * (x + y)))


def test_periodic_conservation():
    """Sum over cells of rho, j, e is exact: the collision conserves them and
    the Lax-Wendroff differences telescope on a periodic grid."""
    ny, nx = 12, 16
    p = mrt.Params(gamma=1.3, s=rates(300, 600, 900, 5e3), dt=1e-4, dx=1 / nx, dy=1 / ny)
    rho = 1 + _smooth_field(ny, nx, 0.2)
    T = 1 - _smooth_field(ny, nx, 0.1).T.reshape(ny, nx) * 0.5
    f = mrt.init_populations(rho, _smooth_field(ny, nx, 0.3), -_smooth_field(ny, nx, 0.2), T, p)
    f = f * (1 + 0.01 * RNG.standard_normal(f.shape))      # off equilibrium
    M = mrt.transformation_matrix()
    before = (M[:4] @ f.reshape(16, -1)).sum(axis=1)
    f = mrt.run(f, p, 30)
    after = (M[:4] @ f.reshape(16, -1)).sum(axis=1)
    np.testing.assert_allclose(after, before, rtol=1e-13, atol=1e-13)


def test_free_streaming_moves_each_population_at_its_velocity():
    """With every s_k = 0, each population obeys df/dt + v.grad f = 0.  The
    Lax-Wendroff update then moves the centroid of f_i by exactly
    v_i dt per step and keeps its variance (both are exact properties of the
    three-point Lax-Wendroff difference)."""
    ny, nx = 40, 48
    dx, dy, dt = 0.01, 0.02, 2e-4
    p = mrt.Params(gamma=1.4, s=np.zeros(16), dt=dt, dx=dx, dy=dy)
    y, x = np.meshgrid(np.arange(ny) * dy, np.arange(nx) * dx, indexing="ij")
    bump = np.exp(-((x - 0.24) ** 2) / 0.001 - ((y - 0.4) ** 2) / 0.003)
    f = np.broadcast_to(bump, (16, ny, nx)).copy()
    n = 25
    g = mrt.run(f, p, n)
    vx, vy, _ = mrt.velocity_set()
    for i in range(16):
        m0 = g[i].sum()
        np.testing.assert_allclose(m0, f[i].sum(), rtol=1e-13)
        cx0, cy0 = (x * f[i]).sum() / m0, (y * f[i]).sum() / m0
        cx1, cy1 = (x * g[i]).sum() / m0, (y * g[i]).sum() / m0
        assert cx1 - cx0 == pytest.approx(vx[i] * dt * n, abs=1e-12)
        assert cy1 - cy0 == pytest.approx(vy[i] * dt * n, abs=1e-12)
        var0 = ((x - cx0) ** 2 * f[i]).sum() / m0
        var1 = ((x - cx1) ** 2 * g[i]).sum() / m0
        assert var1 == pytest.approx(var0, abs=1e-12)


def _sod(nx, gamma=1.4, flip=False, nsteps=None, tend=0.1, dt=None, s=None, ny=1):
    dx = 1.0 / nx
    dt = dt or 0.1 * dx / 6.0
    L, R = (1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.8)
    if flip:
        L, R = R, L
    p = mrt.Params(gamma=gamma, s=s if s is not None else rates(0.5 / dt, 0.5 / dt, 0.5 / dt, 1 / dt),
                   dt=dt, dx=dx, dy=dx,
                   bc=(mrt.BC_EQ, mrt.BC_EQ, mrt.BC_PERIODIC, mrt.BC_PERIODIC),
                   side_state=(L, R, L, L))
    x = (np.arange(nx) + 0.5) * dx
    left = np.broadcast_to(x < 0.5, (ny, nx))
    rho = np.where(left, L[0], R[0])
    T = np.where(left, L[3], R[3])
    f = mrt.init_populations(rho, 0 * rho, 0 * rho, T, p)
    n = nsteps or int(round(tend / dt))
    f = mrt.run(f, p, n)
    return x, n * dt, p, f


def test_mirror_symmetry():
    """The velocity set is closed under x -> -x, so the mirrored tube gives
    the mirrored solution."""
    s = rates(500, 1000, 710, 1e5)
    x, t, p, f = _sod(80, nsteps=60, dt=1e-5, s=s)
    _, _, _, g = _sod(80, flip=True, nsteps=60, dt=1e-5, s=s)
    r1, u1, _, T1 = mrt.macroscopic(f, p.b)
    r2, u2, _, T2 = mrt.macroscopic(g, p.b)
    np.testing.assert_allclose(r1, r2[:, ::-1], rtol=1e-12)
    np.testing.assert_allclose(u1, -u2[:, ::-1], rtol=0, atol=1e-12)
    np.testing.assert_allclose(T1, T2[:, ::-1], rtol=1e-12)


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0])
@pytest.mark.parametrize("T", [0.5, 2.0])
def test_sound_speed(gamma, T):
    """Section (a): a pressure ratio 1 + 1e-10 at equal T splits into two
    acoustic fronts moving at c_s = sqrt(gamma T).  The measured speed
    converges to c_s under refinement."""
    errs = []
    for nx in (200, 400):
        dx = 1.0 / nx
        dt = 0.3 * dx / 6.0
        hi, lo = (1 + 1e-10, 0.0, 0.0, T), (1.0, 0.0, 0.0, T)
        p = mrt.Params(gamma=gamma, s=rates(1 / dt, 1 / dt, 1 / dt, 1 / dt), dt=dt, dx=dx, dy=dx,
                       bc=(mrt.BC_EQ, mrt.BC_EQ, mrt.BC_PERIODIC, mrt.BC_PERIODIC),
                       side_state=(hi, lo, lo, lo))
        x = (np.arange(nx) + 0.5) * dx
        rho = np.where(x < 0.5, 1 + 1e-10, 1.0)[None, :]
        f = mrt.init_populations(rho, 0 * rho, 0 * rho, T + 0 * rho, p)
        cs = np.sqrt(gamma * T)
        n = int(round(0.3 / cs / dt))
        f = mrt.run(f, p, n)
        r, _, _, TT = mrt.macroscopic(f, p.b)
        pp = ((r * TT)[0] - T) / (1e-10 * T)
        i = np.where(pp > 0.25)[0].max()
        xf = x[i] + (pp[i] - 0.25) / (pp[i] - pp[i + 1]) * dx
        errs.append(abs((xf - 0.5) / (n * dt) / cs - 1.0))
    assert errs[1] < 0.015
    assert errs[1] < 0.75 * errs[0]


def test_sod_matches_exact_riemann_and_converges():
    """Section (b): shock tube against the exact Riemann solution; the L1
    error of rho, u, p falls under refinement."""
    # viscosity and time step scale with dx; s_10..16 dt = 1
    s_of = lambda nx: rates(500 * nx / 400, 1000 * nx / 400, 710 * nx / 400, 1e5 * nx / 400)
    errs = []
    for nx in (100, 200, 400):
        x, t, p, f = _sod(nx, dt=1e-5 * 400 / nx, s=s_of(nx), tend=0.1)
        r, u, _, T = mrt.macroscopic(f, p.b)
        er, eu, ep = riemann.sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), 1.4, (x - 0.5) / t)
        errs.append([np.mean(np.abs(r[0] - er)), np.mean(np.abs(u[0] - eu)),
                     np.mean(np.abs(r[0] * T[0] - ep))])
    errs = np.array(errs)
    assert np.all(errs[1] < 0.8 * errs[0]) and np.all(errs[2] < 0.8 * errs[1])
    assert errs[2, 0] < 0.012 and errs[2, 1] < 0.02 and errs[2, 2] < 0.01


def _wave_decay(mode, s7, Pr, nx=32, sdt=0.02, tend=1.0, U=1e-3, T=1.0):
    dx = 1.0 / nx
    dt = sdt / s7
    p = mrt.Params(gamma=1.4, s=rates(s7, s7, Pr * s7, min(1 / dt, 50 * s7)), dt=dt, dx=dx, dy=dx)
    x = (np.arange(nx) + 0.5) * dx
    sn = np.sin(2 * np.pi * x)[None, :]
    if mode == "shear":
        f = mrt.init_populations(1 + 0 * sn, 0 * sn, U * sn, T + 0 * sn, p)
    else:   # entropy wave: T modulated at constant pressure
        f = mrt.init_populations(1 / (1 + U * sn), 0 * sn, 0 * sn, T * (1 + U * sn), p)
    n = int(round(tend / dt))
    r, ux, uy, TT = mrt.macroscopic(mrt.run(f, p, n), p.b)
    q = uy if mode == "shear" else (TT - T) / T
    amp = 2 * np.mean(q * sn) / U
    return -np.log(amp) / (n * dt) / (2 * np.pi) ** 2


def test_shear_viscosity():
    """Eqs. (12b)-(12c): kinematic viscosity nu = R T / s_7 (= R T / s_6)."""
    nu = _wave_decay("shear", s7=50.0, Pr=1.0)
    assert nu == pytest.approx(1.0 / 50.0, rel=0.015)


@pytest.mark.parametrize("Pr", [0.5, 2.0])
def test_thermal_diffusivity_sets_prandtl(Pr):
    """Eq. (12d): heat conductivity (b/2+1) R rho R T / s_8, so the thermal
    diffusivity is R T / s_8 and Pr = nu / alpha = s_8 / s_7."""
    alpha = _wave_decay("entropy", s7=50.0, Pr=Pr)
    nu = _wave_decay("shear", s7=50.0, Pr=Pr)
    assert alpha == pytest.approx(1.0 / (Pr * 50.0), rel=0.03)
    assert nu / alpha == pytest.approx(Pr, rel=0.03)


@pytest.mark.slow
def test_couette_energy_balance_follows_eq_12d():
    """Steady thermal Couette flow.  In Eq. (12d) the viscous-heating term
    and the conduction term both carry 1/s_8 (= 1/s_9), so in the core of a
    symmetric Couette flow T + u^2/(b+2) is constant whatever Pr; the
    textbook Navier-Stokes balance would instead keep T + Pr u^2/(b+2)
    constant.  At Pr = 2 the oracle must follow the former."""
    ny, s7, Pr, U, T0 = 16, 20.0, 2.0, 0.4, 1.0
    dy, dt = 1.0 / ny, 1e-3
    p = mrt.Params(gamma=1.4, s=rates(s7, s7, Pr * s7, 1000.0), dt=dt, dx=dy, dy=dy,
                   bc=(mrt.BC_PERIODIC, mrt.BC_PERIODIC, mrt.BC_EQ, mrt.BC_EQ),
                   side_state=((1.0, 0, 0, T0), (1.0, 0, 0, T0), (1.0, -U / 2, 0, T0), (1.0, U / 2, 0, T0)))
    y = (np.arange(ny) + 0.5) * dy
    u0 = 0.6 * U * (y - 0.5)
    T_init = T0 + (0.09 * U * U - u0 ** 2) / (p.b + 2)
    f = mrt.init_populations((T0 / T_init)[:, None], u0[:, None], 0 * u0[:, None], T_init[:, None], p)
    f = mrt.run(f, p, int(round(6 / (T0 / s7 * np.pi ** 2) / dt)))
    _, u, _, T = mrt.macroscopic(f, p.b)
    u, T = u[:, 0], T[:, 0]
    core = slice(ny // 4, 3 * ny // 4)
    spread = lambda a: np.ptp(a[core])
    assert spread(T) > 3e-4
    assert spread(T + u * u / (p.b + 2)) < 0.35 * spread(T)
    assert spread(T + Pr * u * u / (p.b + 2)) > 0.7 * spread(T)


def test_reflecting_ghost_reverses_normal_velocity():
    """Section (d): the ghost carries the mirror cell's state with the normal
    velocity reversed (rho, tangential velocity and T unchanged)."""
    p = mrt.Params(gamma=1.4, s=np.zeros(16), dt=1e-4, dx=0.1, dy=0.1,
                   bc=(mrt.BC_REFLECT, mrt.BC_OUTFLOW, mrt.BC_REFLECT, mrt.BC_EQ))
    rho = 1 + 0.3 * RNG.random((3, 4))
    ux, uy = RNG.standard_normal((3, 4)) * 0.3, RNG.standard_normal((3, 4)) * 0.3
    T = 0.5 + RNG.random((3, 4))
    g = mrt.fill_ghosts(mrt.init_populations(rho, ux, uy, T, p), p)
    r, u, v, t = mrt.macroscopic(g[:, 1:-1, 0], p.b)          # x-lo ghost column
    np.testing.assert_allclose((r, u, v, t), (rho[:, 0], -ux[:, 0], uy[:, 0], T[:, 0]), rtol=1e-12, atol=1e-13)
    r, u, v, t = mrt.macroscopic(g[:, 0, 1:-1], p.b)          # y-lo ghost row
    np.testing.assert_allclose((r, u, v, t), (rho[0], ux[0], -uy[0], T[0]), rtol=1e-12, atol=1e-13)
    np.testing.assert_array_equal(g[:, 1:-1, -1], g[:, 1:-1, -2])   # outflow copies


def test_window_evaluation_matches_full_grid():
    ny, nx, k = 20, 24, 3
    p = mrt.Params(gamma=1.4, s=rates(500, 1000, 710, 1e4), dt=2e-5, dx=1 / 64, dy=1 / 64,
                   bc=(mrt.BC_EQ, mrt.BC_OUTFLOW, mrt.BC_REFLECT, mrt.BC_REFLECT),
                   side_state=((1.5, 0.3, 0.0, 1.2),) * 4)
    rho = 1 + _smooth_field(ny, nx, 0.2)
    T = 1 + _smooth_field(ny, nx, 0.1)
    ux, uy = _smooth_field(ny, nx, 0.3), _smooth_field(ny, nx, -0.2)
    full = mrt.run(mrt.init_populations(rho, ux, uy, T, p), p, k)
    for x0, x1, y0, y1 in ((0, 10, 0, 9), (7, 20, 5, 15), (14, 24, 11, 20)):
        win, (a, b, c, d) = mrt.evolve_window(rho, ux, uy, T, p, x0, x1, y0, y1, k)
        ok = np.isfinite(win).all(axis=0)
        assert ok.sum() > 0
        np.testing.assert_allclose(win[:, ok], full[:, c:d, a:b][:, ok], rtol=1e-13, atol=1e-14)
        # cells at least k away from an interior window side are known
        iy0 = 0 if y0 == 0 else k
        iy1 = (d - c) if y1 == ny else (d - c) - k
        ix0 = 0 if x0 == 0 else k
        ix1 = (b - a) if x1 == nx else (b - a) - k
        assert ok[iy0:iy1, ix0:ix1].all()


def test_linear_stability_interval():
    """The paper asks s_5..s_16 in [0, 1/dt] for linear stability; a rest
    state is stable inside that interval and unstable well outside it."""
    st = (1.0, 0.0, 0.0, 1.0)
    dt = 1e-4
    inside = mrt.Params(gamma=1.4, s=rates(0.5 / dt, 1 / dt, 1 / dt, 1 / dt), dt=dt, dx=0.01, dy=0.01)
    outside = mrt.Params(gamma=1.4, s=rates(3 / dt, 3 / dt, 3 / dt, 3 / dt), dt=dt, dx=0.01, dy=0.01)
    assert stability.max_amplification(st, inside, 17) <= 1 + 1e-12
    assert stability.max_amplification(st, outside, 17) > 1.5


@pytest.mark.parametrize("reading", ["unsplit", "split"])
def test_small_perturbations_follow_the_amplification_matrix(reading):
    """The linear-stability tool is the scheme's own linearisation: a small
    Fourier perturbation of a uniform moving equilibrium, advanced by the
    nonlinear oracle step (unsplit, or the collide-then-convect option),
    equals G(theta)^N applied to it (G from oracle/stability.py), to first
    order in the amplitude."""
    n, N, eps = 16, 25, 1e-6
    p = mrt.Params(gamma=1.4, s=rates(3e3, 6e3, 0.71, 8e3), dt=1e-4, dx=1.0 / n, dy=1.0 / n,
                   split=(reading == "split"))
    base = (1.0, 0.3, -0.2, 0.9)
    f0 = mrt.feq(*base, p.b).reshape(16, 1, 1)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(16)
    kx, ky = 1, 2
    tx, ty = 2 * np.pi * kx / n, 2 * np.pi * ky / n
    Y, X = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    phase = tx * X + ty * Y
    f = f0 + eps * v.reshape(16, 1, 1) * np.cos(phase)
    for _ in range(N):
        f = mrt.step(f, p)
    # Fourier component at (kx, ky): the cosine's e^{+i phase} half
    got = 2.0 * np.mean((f - f0) * np.exp(-1j * phase), axis=(1, 2)) / eps
    G = stability.amplification_matrix(base, p, tx, ty, reading)
    want = np.linalg.matrix_power(G, N) @ v
    assert np.allclose(got, want, rtol=0, atol=1e-5 * np.abs(want).max())
    # and the transfer is not trivial: the mode changed over the run
    assert np.abs(want - v).max() > 1e-2 * np.abs(v).max()


def test_reading_amplifications_reduce_to_their_textbook_factors():
    """Every reading of the time/space passage in the stability tool: with
    theta = 0 (no convection) each mode of the linear collision K = dt J_C,
    eigenvalue k, is multiplied by the scalar factor of its time integrator
    (forward Euler 1 - k, split the same, Taylor 1 - k + k^2/2, Crank-Nicolson
    (1 - k/2)/(1 + k/2), exact e^-k); with every rate zero (no collision) each
    reading is the Lax-Wendroff symbol 1 - i c sin(theta) + c^2 (cos(theta) - 1)
    per population."""
    st = (1.1, 0.4, -0.3, 0.8)
    p = mrt.Params(gamma=1.4, s=rates(3e3, 6e3, 0.71, 8e3), dt=1e-4, dx=1e-3, dy=1e-3)
    from oracle.adjoint import collision_jacobian
    f0 = mrt.feq(*st, p.b).reshape(16, 1, 1)
    k = np.linalg.eigvals(p.dt * collision_jacobian(f0, p)[:, :, 0, 0])
    factors = {"unsplit": 1 - k, "split": 1 - k, "rhs_taylor": 1 - k + k * k / 2,
               "trapezoid": (1 - k / 2) / (1 + k / 2), "exp_collision": np.exp(-k)}
    for reading in stability.READINGS:
        ev = np.linalg.eigvals(stability.amplification_matrix(st, p, 0.0, 0.0, reading))
        want = factors[reading]
        # match the two spectra as multisets
        d = np.abs(ev[:, None] - want[None, :])
        assert np.max(np.min(d, axis=1)) < 1e-9 and np.max(np.min(d, axis=0)) < 1e-9, reading
    p0 = mrt.Params(gamma=1.4, s=np.zeros(16), dt=1e-4, dx=1e-3, dy=2e-3)
    vx, vy, _ = mrt.velocity_set()
    cx, cy = vx * p0.dt / p0.dx, vy * p0.dt / p0.dy
    tx, ty = 0.7, -1.9
    sym = (1 - 1j * cx * np.sin(tx) + cx ** 2 * (np.cos(tx) - 1)
           - 1j * cy * np.sin(ty) + cy ** 2 * (np.cos(ty) - 1))
    for reading in stability.READINGS:
        G = stability.amplification_matrix(st, p0, tx, ty, reading)
        assert np.allclose(G, np.diag(sym), rtol=0, atol=1e-13), reading
