"""Pins of the oracle's two alternative readings of the time/space
discretisation: the collide-then-stream split and the nine-point 2D
Lax-Wendroff stencil (mixed-derivative term)."""
import numpy as np
import pytest

from oracle import mrt
from oracle.adjoint import collision_jacobian

N = 16


def _params(**kw):
    base = dict(gamma=1.4, s=[0.0] * 4 + [3e3] * 12, dt=1e-4, dx=1.0 / 32, dy=1.0 / 24)
    base.update(kw)
    return mrt.Params(**base)


def _textbook_lw_symbol(cx, cy, tx, ty, cross):
    """Amplification of the Lax-Wendroff scheme for u_t + a u_x + b u_y = 0
    (Courant numbers cx, cy): second-order Taylor series in time with
    central differences; the mixed term -cx cy sin(tx) sin(ty) only in the
    full two-dimensional scheme."""
    g = 1.0 - 1j * (cx * np.sin(tx) + cy * np.sin(ty)) - cx ** 2 * (1 - np.cos(tx)) - cy ** 2 * (1 - np.cos(ty))
    if cross:
        g = g - cx * cy * np.sin(tx) * np.sin(ty)
    return g


@pytest.mark.parametrize("cross", [False, True])
def test_free_streaming_symbol_is_the_textbook_lax_wendroff(cross):
    """With every rate zero the step is pure convection of each population:
    one oracle step applied to a Fourier mode on a periodic grid multiplies
    it by the textbook symbol, the mixed term included with lw_cross."""
    nx, ny = 32, 24
    p = _params(s=[0.0] * 16, lw_cross=cross, dt=2e-3)
    kx, ky = 3, 5
    x = np.arange(nx)
    y = np.arange(ny)
    Y, X = np.meshgrid(y, x, indexing="ij")
    tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
    phase = tx * X + ty * Y
    eps = 1e-3
    fc = np.ones((N, ny, nx)) + eps * np.cos(phase)
    fs = np.ones((N, ny, nx)) + eps * np.sin(phase)
    z = (mrt.step(fc, p) - 1.0 + 1j * (mrt.step(fs, p) - 1.0)) / eps
    G = z / np.exp(1j * phase)
    cx, cy = mrt.courant_numbers(p)
    for i in range(N):
        want = _textbook_lw_symbol(cx[i, 0, 0], cy[i, 0, 0], tx, ty, cross)
        assert np.allclose(G[i], want, rtol=0, atol=1e-12), i


def test_nine_point_stencil_is_second_order_for_diagonal_transport():
    """Free streaming of a smooth periodic bump in a diagonal population:
    the nine-point scheme converges at second order, the five-point one
    (which misses the mixed derivative of the Taylor series) at first
    order, at a fixed Courant number."""
    def err(n, cross):
        p = mrt.Params(gamma=1.4, s=[0.0] * 16, dx=1.0 / n, dy=1.0 / n, dt=0.3 / n,
                       lw_cross=cross)     # Courant number 0.64 for this population
        x = (np.arange(n) + 0.5) / n
        Y, X = np.meshgrid(x, x, indexing="ij")
        bump = lambda X, Y: np.exp(np.cos(2 * np.pi * X) + np.sin(2 * np.pi * Y))
        f = np.ones((N, n, n))
        i = 12                              # shell 4, velocity (3/sqrt2)(+1, +1)
        vx, vy, _ = mrt.velocity_set()
        f[i] = bump(X, Y)
        steps = int(round(0.2 / p.dt))
        for _ in range(steps):
            f = mrt.step(f, p)
        t = steps * p.dt
        return np.max(np.abs(f[i] - bump(X - vx[i] * t, Y - vy[i] * t)))
    e9 = [err(n, True) for n in (32, 64)]
    e5 = [err(n, False) for n in (32, 64)]
    assert 3.5 < e9[0] / e9[1] < 4.5          # second order
    assert 1.7 < e5[0] / e5[1] < 2.4          # first order
    assert e9[1] < 0.2 * e5[1]


@pytest.mark.parametrize("tx,ty", [(0.4, -1.1), (2.0, 0.7)])
def test_split_step_is_stream_after_collide_in_fourier_space(tx, ty):
    """Linearised about a uniform equilibrium, one split step multiplies a
    Fourier mode by diag(textbook symbol) (I - dt J), J the collision
    Jacobian; the unsplit step by diag(symbol) - dt J."""
    nx, ny = 20, 20
    kx, ky = int(round(tx * nx / (2 * np.pi))), int(round(ty * ny / (2 * np.pi)))
    tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
    state = (1.1, 0.3, -0.2, 0.9)
    for split in (False, True):
        p = _params(split=split, dx=1.0 / nx, dy=1.0 / ny, dt=1e-4)
        f0 = mrt.feq(*state, p.b).reshape(N, 1, 1)
        J = collision_jacobian(f0, p)[:, :, 0, 0]
        cx, cy = mrt.courant_numbers(p)
        L = np.diag([_textbook_lw_symbol(cx[i, 0, 0], cy[i, 0, 0], tx, ty, False) for i in range(N)])
        want = L @ (np.eye(N) - p.dt * J) if split else L - p.dt * J
        Y, X = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        phase = tx * X + ty * Y
        eps = 1e-6
        got = np.zeros((N, N), dtype=complex)
        for j in range(N):
            e = np.zeros((N, 1, 1)); e[j] = 1.0
            # central differences: the response is linear to O(eps^2)
            dc = mrt.step(f0 + eps * e * np.cos(phase), p) - mrt.step(f0 - eps * e * np.cos(phase), p)
            ds = mrt.step(f0 + eps * e * np.sin(phase), p) - mrt.step(f0 - eps * e * np.sin(phase), p)
            z = (dc + 1j * ds) / (2 * eps)
            got[:, j] = (z / np.exp(1j * phase))[:, 3, 5]
        # (the other composition differs by ~3e-3 of the scale)
        assert np.allclose(got, want, rtol=0, atol=1e-9 * np.abs(want).max()), split


@pytest.mark.parametrize("split,cross", [(True, False), (False, True), (True, True)])
def test_variants_conserve_on_periodic_grids(split, cross):
    rng = np.random.default_rng(4)
    n = 12
    p = _params(split=split, lw_cross=cross, dx=1.0 / n, dy=1.0 / n)
    rho = 1 + 0.1 * rng.random((n, n))
    T = 1 + 0.1 * rng.random((n, n))
    u = 0.2 * rng.standard_normal((2, n, n))
    f = mrt.init_populations(rho, u[0], u[1], T, p) * (1 + 0.01 * rng.standard_normal((N, n, n)))
    m0 = mrt.kinetic_moments(f)[:4].sum(axis=(1, 2))
    g = mrt.run(f, p, 20)
    m1 = mrt.kinetic_moments(g)[:4].sum(axis=(1, 2))
    assert np.allclose(m0, m1, rtol=1e-13, atol=1e-13)


def test_uniform_state_sees_only_the_collision():
    """No gradients: both readings reduce to f - dt C(f) (the collision is
    applied exactly once), whatever the stencil."""
    rng = np.random.default_rng(6)
    p0 = _params()
    f1 = mrt.feq(1.0, 0.2, 0.1, 1.0, p0.b) * (1 + 0.05 * rng.standard_normal(N))
    f = np.broadcast_to(f1.reshape(N, 1, 1), (N, 6, 7)).copy()
    want = f - p0.dt * mrt.collision(f, p0)
    for split in (False, True):
        for cross in (False, True):
            p = _params(split=split, lw_cross=cross)
            assert np.allclose(mrt.step(f, p), want, rtol=0, atol=1e-14)


def test_corner_ghosts_keep_a_diagonal_mirror_symmetry():
    """Reflecting walls on all four sides of a square grid and a field
    symmetric under the swap x <-> y (velocity components swapped too): the
    nine-point step keeps the symmetry, corners included, so the corner
    ghosts treat the two axes alike."""
    n = 10
    p = _params(lw_cross=True, dx=1.0 / n, dy=1.0 / n, bc=(mrt.BC_REFLECT,) * 4)
    rng = np.random.default_rng(8)
    a = rng.random((n, n))
    sym = a + a.T
    rho = 1 + 0.1 * sym
    T = 1 + 0.05 * sym
    ux = 0.1 * rng.random((n, n))
    uy = ux.T.copy()
    f = mrt.init_populations(rho, ux, uy, T, p)
    g = mrt.run(f, p, 5)
    r, u, v, t = mrt.macroscopic(g, p.b)
    assert np.allclose(r, r.T, rtol=0, atol=1e-13)
    assert np.allclose(u, v.T, rtol=0, atol=1e-13)
    assert np.allclose(t, t.T, rtol=0, atol=1e-13)
    # and the corner cells did see the corner ghosts: without them (NaN) the
    # corners would be undefined
    assert np.isfinite(g).all()
