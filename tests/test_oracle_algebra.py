"""Pins of the oracle's algebra: velocity set, M, Minv, equilibrium, collision.

Each test checks the oracle against something other than itself: exact
symbolic linear algebra, the continuous Maxwellian moments that the paper's
seven-moment relations express, or structural identities of Eq. (3).
"""
import numpy as np
import pytest
import sympy as sp

from oracle import mrt

RNG = np.random.default_rng(1234)


def test_velocity_shells():
    vx, vy, eta = mrt.velocity_set()
    speed = np.hypot(vx, vy)
    # four energy levels v = 1, 6, 2, 3 (section "Construction")
    np.testing.assert_allclose(speed, [1] * 4 + [6] * 4 + [2] * 4 + [3] * 4, rtol=0, atol=1e-15)
    # each shell is closed under the 90-degree rotation (x, y) -> (-y, x)
    for k in range(4):
        sl = slice(4 * k, 4 * k + 4)
        shell = {(round(a, 12), round(b, 12)) for a, b in zip(vx[sl], vy[sl])}
        rot = {(round(-b, 12), round(a, 12)) for a, b in shell}
        assert shell == rot
    np.testing.assert_array_equal(eta, [2.5] * 4 + [0.0] * 12)


def _sym_velocities():
    r2 = sp.sqrt(2)
    axis = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    diag = [(1, 1), (-1, 1), (-1, -1), (1, -1)]
    v = ([(sp.Integer(a), sp.Integer(b)) for a, b in axis]
         + [(6 * sp.Integer(a), 6 * sp.Integer(b)) for a, b in axis]
         + [(r2 * a, r2 * b) for a, b in diag]
         + [(3 * a / r2, 3 * b / r2) for a, b in diag])
    eta = [sp.Rational(5, 2)] * 4 + [sp.Integer(0)] * 12
    return v, eta


def test_inverse_is_exact():
    """Minv equals the exact symbolic inverse; M Minv = I to rounding."""
    M = mrt.transformation_matrix()
    Minv = mrt.inverse_matrix()
    np.testing.assert_allclose(M @ Minv, np.eye(16), rtol=0, atol=2e-14)
    Ms = sp.Matrix(16, 16, lambda r, c: sp.nsimplify(M[r, c], [sp.sqrt(2)]))
    Minv_exact = np.array(Ms.inv().evalf(30), dtype=float)
    np.testing.assert_allclose(Minv, Minv_exact, rtol=0, atol=1e-14)
    # a few exact entries (1-based [row, col]); rationals because they only
    # involve the scalar shell moments
    exact = {(1, 4): sp.Rational(1, 25), (1, 5): sp.Rational(-1, 25),
             (1, 6): sp.Rational(36, 115), (1, 16): sp.Rational(-1, 115),
             (5, 1): sp.Rational(1, 96), (5, 6): sp.Rational(-29, 16560),
             (9, 1): sp.Rational(81, 160), (13, 1): sp.Rational(-4, 15)}
    for (r, c), val in exact.items():
        assert Ms.inv()[r - 1, c - 1] == val
        assert Minv[r - 1, c - 1] == pytest.approx(float(val), abs=1e-15)
    assert np.count_nonzero(np.abs(M) > 1e-12) == 176
    assert np.count_nonzero(np.abs(Minv) > 1e-12) == 172


def _maxwellian_moments(rho, ux, uy, T, b):
    """The right-hand sides of the seven moment relations: moments of the
    continuous 2D Maxwellian with (b-2) extra degrees of freedom carried by
    eta^2 (each extra dof holds T/2 of internal energy), R = 1."""
    u = (ux, uy)
    u2 = ux * ux + uy * uy
    d = lambda a, c: 1.0 if a == c else 0.0
    out = {"1": rho}
    for a in range(2):
        out[f"v{a}"] = rho * u[a]
        out[f"ev{a}"] = rho * u[a] * ((b + 2) * T + u2)
        for c in range(2):
            out[f"v{a}v{c}"] = rho * (T * d(a, c) + u[a] * u[c])
            out[f"ev{a}v{c}"] = (rho * T * ((b + 2) * T + u2) * d(a, c)
                                 + rho * u[a] * u[c] * ((b + 4) * T + u2))
            for e in range(2):
                out[f"v{a}v{c}v{e}"] = rho * (T * (u[a] * d(c, e) + u[c] * d(a, e) + u[e] * d(a, c))
                                             + u[a] * u[c] * u[e])
    out["e"] = rho * (b * T + u2)
    return out


def _discrete_moments(f, eta0=2.5):
    vx, vy, eta = mrt.velocity_set(eta0)
    v = (vx, vy)
    eps = vx * vx + vy * vy + eta * eta
    out = {"1": f.sum(), "e": (eps * f).sum()}
    for a in range(2):
        out[f"v{a}"] = (v[a] * f).sum()
        out[f"ev{a}"] = (eps * v[a] * f).sum()
        for c in range(2):
            out[f"v{a}v{c}"] = (v[a] * v[c] * f).sum()
            out[f"ev{a}v{c}"] = (eps * v[a] * v[c] * f).sum()
            for e in range(2):
                out[f"v{a}v{c}v{e}"] = (v[a] * v[c] * v[e] * f).sum()
    return out


@pytest.mark.parametrize("seed", range(40))
def test_seven_moment_relations(seed):
    """f^eq = Minv fhat^eq satisfies every moment relation to rounding."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.1, 5.0)
    T = rng.uniform(0.05, 10.0)
    ma = rng.uniform(0.0, 5.0)
    ang = rng.uniform(0, 2 * np.pi)
    ux, uy = ma * np.sqrt(T) * np.cos(ang), ma * np.sqrt(T) * np.sin(ang)
    gamma = rng.uniform(1.05, 2.0)
    b = mrt.b_from_gamma(gamma)
    f = mrt.feq(rho, ux, uy, T, b)
    want = _maxwellian_moments(rho, ux, uy, T, b)
    got = _discrete_moments(f)
    scale = np.sum(np.abs(f)) * (1 + 36.0) ** 2
    for key, val in want.items():
        assert abs(got[key] - val) <= 1e-13 * scale, key


def test_equilibrium_solves_velocity_space_constraints_exactly():
    """Solve the 16 moment constraints for f directly (exact arithmetic) and
    compare with Minv fhat^eq: an independent route to the same f^eq."""
    v, eta = _sym_velocities()
    rho, ux, uy, T, b = sp.Integer(1), sp.Rational(3, 10), sp.Rational(-1, 5), sp.Integer(1), sp.Integer(5)
    rhs = _maxwellian_moments(rho, ux, uy, T, b)
    keys = ["1", "v0", "v1", "e", "v0v0", "v0v1", "v1v1", "ev0", "ev1",
            "v0v0v0", "v0v0v1", "v0v1v1", "v1v1v1", "ev0v0", "ev0v1", "ev1v1"]

    def mono(key, i):
        vxi, vyi = v[i]
        comps = {"0": vxi, "1": vyi}
        eps = vxi ** 2 + vyi ** 2 + eta[i] ** 2
        if key == "1":
            return sp.Integer(1)
        if key == "e":
            return eps
        val = sp.Integer(1)
        rest = key
        if rest.startswith("e"):
            val = eps
            rest = rest[1:]
        for ch in rest.split("v")[1:]:
            val = val * comps[ch]
        return val

    A = sp.Matrix(16, 16, lambda r, c: mono(keys[r], c))
    y = sp.Matrix([sp.nsimplify(rhs[k]) for k in keys])
    f_exact = A.LUsolve(y)
    f_exact = np.array([float(sp.nsimplify(x).evalf(30)) for x in f_exact])
    f = mrt.feq(1.0, 0.3, -0.2, 1.0, 5.0)
    np.testing.assert_allclose(f, f_exact, rtol=0, atol=2e-15)
    # rest state, b = 5: shell values 3/25, 79/28800, 553/3200, -41/900
    f0 = mrt.feq(1.0, 0.0, 0.0, 1.0, 5.0)
    want = np.repeat([3 / 25, 79 / 28800, 553 / 3200, -41 / 900], 4)
    np.testing.assert_allclose(f0, want, rtol=0, atol=1e-15)


def test_collision_conserves_rho_j_e():
    """fhat_1..4 are collision invariants: rows 1-4 of M C vanish."""
    p = mrt.Params(gamma=1.4, s=RNG.uniform(0, 1e4, 16), dt=1e-4)
    f = mrt.feq(1.0, 0.2, 0.1, 1.0, p.b)[:, None] * (1 + 0.05 * RNG.standard_normal((16, 50)))
    C = mrt.collision(f, p)
    MC = mrt.transformation_matrix() @ C
    scale = np.abs(mrt.transformation_matrix()).max() * np.abs(C).max()
    assert np.abs(MC[:4]).max() < 1e-13 * scale


def test_collision_is_diagonal_in_moment_space():
    """M C = diag(s) (M f - fhat^eq): each moment relaxes at its own rate
    (Eq. 3 and the relaxation matrix S_hat = diag(s_1..s_N))."""
    p = mrt.Params(gamma=5 / 3, s=RNG.uniform(0, 1e3, 16), dt=1e-4)
    f = mrt.feq(0.7, -0.3, 0.4, 1.3, p.b)[:, None] * (1 + 0.1 * RNG.standard_normal((16, 20)))
    M = mrt.transformation_matrix()
    m = M @ f
    meq = mrt.equilibrium_moments(m[0], m[1], m[2], m[3], p.b)
    for k in range(4, 16):
        s = np.zeros(16)
        s[k] = 7.0
        pk = mrt.Params(gamma=p.gamma, s=s, dt=p.dt)
        MC = M @ mrt.collision(f, pk)
        want = np.zeros_like(MC)
        want[k] = 7.0 * (m[k] - meq[k])
        np.testing.assert_allclose(MC, want, rtol=0, atol=1e-10 * np.abs(m).max())


def test_bgk_limit():
    """All rates equal to 1/tau: C = (f - f^eq)/tau (text after Eq. 3)."""
    tau = 2.5e-3
    p = mrt.Params(gamma=1.4, s=[1 / tau] * 16, dt=1e-4)
    f = mrt.feq(1.2, 0.1, -0.3, 0.8, p.b)[:, None] * (1 + 0.1 * RNG.standard_normal((16, 30)))
    rho, ux, uy, T = mrt.macroscopic(f, p.b)
    want = (f - mrt.feq(rho, ux, uy, T, p.b)) / tau
    np.testing.assert_allclose(mrt.collision(f, p), want, rtol=0, atol=1e-9 * np.abs(want).max())


def test_collision_vanishes_at_equilibrium():
    p = mrt.Params(gamma=1.3, s=RNG.uniform(0, 1e4, 16), dt=1e-4)
    f = mrt.feq(np.array([0.5, 2.0]), np.array([0.4, -1.0]), np.array([0.0, 0.7]),
                np.array([0.6, 2.2]), p.b)
    assert np.abs(mrt.collision(f, p)).max() < 1e-9


def test_macroscopic_roundtrip():
    b = mrt.b_from_gamma(1.4)
    rho, ux, uy, T = 1.7, -0.4, 0.9, 0.35
    got = mrt.macroscopic(mrt.feq(rho, ux, uy, T, b), b)
    np.testing.assert_allclose(got, (rho, ux, uy, T), rtol=1e-13, atol=1e-14)


def test_prandtl_rates():
    s = np.arange(16, dtype=float) + 1.0
    out = mrt.rates_with_prandtl(s, 0.71)
    assert out[7] == out[8] == pytest.approx(0.71 * s[5])
    np.testing.assert_array_equal(np.delete(out, [7, 8]), np.delete(s, [7, 8]))
