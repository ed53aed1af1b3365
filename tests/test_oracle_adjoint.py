"""Pins of the oracle's discrete adjoint (periodic grid).

The adjoint is checked against directional derivatives of the oracle's own
forward step taken independently of it (complex step of ``mrt.step`` and
central finite differences of the loss), not against itself.
"""
import numpy as np
import pytest

from oracle import adjoint, mrt

RNG = np.random.default_rng(11)


def _params(nx=8, ny=6):
    s = np.zeros(16)
    s[4], s[5], s[6], s[7], s[8] = 500.0, 1000.0, 1000.0, 710.0, 710.0
    s[9:] = 1e4
    return mrt.Params(gamma=1.4, s=s, dt=5e-5, dx=1.0 / nx, dy=1.0 / ny)


def _fields(ny, nx, seed):
    rng = np.random.default_rng(seed)
    rho = 1 + 0.05 * rng.standard_normal((ny, nx))
    T = 1 + 0.05 * rng.standard_normal((ny, nx))
    ux = 0.1 * rng.standard_normal((ny, nx))
    uy = 0.1 * rng.standard_normal((ny, nx))
    return rho, ux, uy, T


def test_lax_wendroff_transpose_dot_product():
    p = _params(9, 7)
    u = RNG.standard_normal((16, 7, 9))
    w = RNG.standard_normal((16, 7, 9))
    Lu = mrt.lax_wendroff(mrt.fill_ghosts(u, p), p)
    Ltw = adjoint.lax_wendroff_transpose(w, p)
    assert np.sum(Lu * w) == pytest.approx(np.sum(u * Ltw), rel=1e-13)


def test_adjoint_step_dot_product():
    """<J v, w> = <v, J^T w> with J v from a complex step of mrt.step."""
    p = _params()
    f = mrt.init_populations(*_fields(6, 8, 1), p)
    v = RNG.standard_normal(f.shape)
    w = RNG.standard_normal(f.shape)
    Jv = np.imag(mrt.step(f + 1e-30j * v, p)) / 1e-30
    JTw, _ = adjoint.adjoint_step(w, f, p)
    assert np.sum(Jv * w) == pytest.approx(np.sum(v * JTw), rel=1e-12)


def test_rate_gradient_of_one_step():
    """ds_k = <w, dF/ds_k>; F is linear in s, so a central difference of
    mrt.step in s_k is exact up to rounding."""
    p = _params()
    f = mrt.init_populations(*_fields(6, 8, 2), p) * (1 + 0.01 * RNG.standard_normal((16, 6, 8)))
    w = RNG.standard_normal(f.shape)
    _, ds = adjoint.adjoint_step(w, f, p)
    for k in range(16):
        h = 10.0
        sp_, sm_ = np.array(p.s, dtype=float), np.array(p.s, dtype=float)
        sp_[k] += h
        sm_[k] -= h
        mk = lambda s: mrt.Params(gamma=p.gamma, s=s, dt=p.dt, dx=p.dx, dy=p.dy)
        dF = (mrt.step(f, mk(sp_)) - mrt.step(f, mk(sm_))) / (2 * h)
        assert ds[k] == pytest.approx(np.sum(w * dF), rel=1e-7, abs=1e-13)
    assert np.max(np.abs(ds[:4])) < 1e-12 * np.max(np.abs(ds))


def test_loss_gradient_matches_central_differences():
    ny, nx, n = 6, 8, 6
    p = _params(nx, ny)
    rho0, ux0, uy0, T0 = _fields(ny, nx, 3)
    target = 1 + 0.02 * RNG.standard_normal((ny, nx))

    def loss(r, t, s):
        pp = mrt.Params(gamma=p.gamma, s=s, dt=p.dt, dx=p.dx, dy=p.dy)
        f = mrt.run(mrt.init_populations(r, ux0, uy0, t, pp), pp, n)
        d = f.sum(axis=0) - target
        return 0.5 * np.sum(d * d)

    L, g = adjoint.density_misfit_gradient(rho0, ux0, uy0, T0, target, p, n)
    assert L == pytest.approx(loss(rho0, T0, p.s), rel=1e-13)
    for trial in range(4):
        dr = RNG.standard_normal((ny, nx))
        dT = RNG.standard_normal((ny, nx))
        ds = RNG.standard_normal(16) * np.asarray(p.s)
        eps = 1e-6
        fd = (loss(rho0 + eps * dr, T0 + eps * dT, np.asarray(p.s) + eps * ds)
              - loss(rho0 - eps * dr, T0 - eps * dT, np.asarray(p.s) - eps * ds)) / (2 * eps)
        ad = np.sum(g["rho"] * dr) + np.sum(g["T"] * dT) + np.sum(g["s"] * ds)
        assert ad == pytest.approx(fd, rel=1e-6)
    assert np.max(np.abs(g["s"][:4])) <= 1e-12 * np.max(np.abs(g["s"]))


def test_init_adjoint_all_four_fields_against_central_differences():
    """Every output of init_adjoint, the velocity gradients included, against
    central differences of <lam0, f^0> taken cell by cell from the real-valued
    init_populations: f^0 is local, so moving one field by eps in every cell
    at once changes each cell's own term only.  The fields have distinct,
    non-zero velocities in both directions, so swapped or sign-flipped ux / uy
    gradients fail."""
    ny, nx = 5, 7
    p = _params(nx, ny)
    rho, ux, uy, T = _fields(ny, nx, 7)
    ux = ux + 0.3
    uy = uy - 0.2
    lam0 = RNG.standard_normal((16, ny, nx))
    got = adjoint.init_adjoint(lam0, rho, ux, uy, T, p)
    fields = [rho, ux, uy, T]
    for k, name in enumerate(("rho", "ux", "uy", "T")):
        eps = 1e-6 * max(1.0, float(np.max(np.abs(fields[k]))))
        up = [a.copy() for a in fields]
        dn = [a.copy() for a in fields]
        up[k] = up[k] + eps
        dn[k] = dn[k] - eps
        fd = np.sum(lam0 * (mrt.init_populations(*up, p) - mrt.init_populations(*dn, p)), axis=0) / (2 * eps)
        assert np.max(np.abs(got[k] - fd)) <= 1e-7 * np.max(np.abs(fd)), name
    # the two velocity gradients are different functions of the state
    assert np.max(np.abs(got[1] - got[2])) > 0.1 * np.max(np.abs(got[1]))
