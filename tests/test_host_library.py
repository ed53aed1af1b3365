"""CPU checks of the HIP library's host side (no GPU needed).

The library evaluates its factored moment transform, equilibrium, collision
and per-cell adjoint with the same templates the kernels run; here they are
compared with the oracle's dense Appendix matrix and complex-step Jacobian.
Also: every symbol include/mrtlb.h declares is exported.
"""
import os
import re

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import mrt

lib = pytest.importorskip("paper_1004_5442_amd.lib")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RNG = np.random.default_rng(5)


def test_header_symbols_are_exported():
    text = open(os.path.join(ROOT, "include", "mrtlb.h")).read()
    names = set(re.findall(r"\b(mrt_[a-z_0-9]+)\s*\(", text))
    assert len(names) > 30
    so = lib.raw()
    for n in sorted(names):
        assert hasattr(so, n), n
    assert names == set(lib.EXPORTED)


@pytest.mark.parametrize("which", [0, 1, 2, 3])
def test_factored_transforms_match_dense_matrix(which):
    M = mrt.transformation_matrix()
    mats = {0: M, 1: np.linalg.inv(M), 2: M.T, 3: np.linalg.inv(M).T}
    for _ in range(20):
        x = RNG.standard_normal(16)
        got = lib.host_transform(which, x)
        want = mats[which] @ x
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * max(1.0, np.abs(want).max()))


def test_equilibrium_matches_oracle():
    for _ in range(50):
        gamma = RNG.uniform(1.05, 2.0)
        rho, T = RNG.uniform(0.1, 5), RNG.uniform(0.05, 10)
        ux, uy = RNG.standard_normal(2) * np.sqrt(T) * 2
        got = lib.host_equilibrium(gamma, rho, ux, uy, T)
        want = mrt.feq(rho, ux, uy, T, mrt.b_from_gamma(gamma))
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.abs(want).sum())


def test_collision_matches_oracle():
    for _ in range(50):
        gamma = RNG.uniform(1.1, 1.9)
        b = mrt.b_from_gamma(gamma)
        s = RNG.uniform(0, 1e4, 16)
        dt = 1e-4
        f = mrt.feq(1.0 + RNG.random(), *(RNG.standard_normal(2) * 0.5), 0.5 + RNG.random(), b)
        f = f * (1 + 0.05 * RNG.standard_normal(16))
        got = lib.host_collision(gamma, s, dt, f)
        p = mrt.Params(gamma=gamma, s=s, dt=dt)
        want = dt * mrt.collision(f.reshape(16, 1), p)[:, 0]
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-12 * np.abs(want).max())


def test_cell_adjoint_matches_complex_step_jacobian():
    for _ in range(20):
        gamma = RNG.uniform(1.1, 1.9)
        b = mrt.b_from_gamma(gamma)
        s = RNG.uniform(0, 1e4, 16)
        dt = 1e-4
        f = mrt.feq(1.0 + RNG.random(), *(RNG.standard_normal(2) * 0.5), 0.5 + RNG.random(), b)
        f = f * (1 + 0.05 * RNG.standard_normal(16))
        lam = RNG.standard_normal(16)
        coll, dsk = lib.host_cell_adjoint(gamma, s, dt, f, lam)
        p = mrt.Params(gamma=gamma, s=s, dt=dt)
        J = oadj.collision_jacobian(f.reshape(16, 1), p)[:, :, 0]
        want = dt * J.T @ lam
        np.testing.assert_allclose(coll, want, rtol=0, atol=1e-11 * np.abs(want).max())
        # minus the cell's share of dL/ds: dt (fhat - fhat^eq)_k (Minv^T lam)_k
        _, ds = oadj.adjoint_step(lam.reshape(16, 1, 1), f.reshape(16, 1, 1),
                                  mrt.Params(gamma=gamma, s=s, dt=dt, dx=1.0, dy=1.0))
        np.testing.assert_allclose(-dsk, ds, rtol=0, atol=1e-11 * np.abs(ds).max())


def _fp32_conserved_exact(f32):
    """Exact rational rho, jx, jy, e of FP32 populations with the FP32 values
    of the Appendix rows m1..m4 (the oracle's dense matrix)."""
    from fractions import Fraction
    M = mrt.transformation_matrix()
    F = [Fraction(float(x)) for x in f32]
    return [sum(Fraction(float(np.float32(M[r, i]))) * F[i] for i in range(16)) for r in range(4)]


def _fp32_cases(rng, n):
    for _ in range(n):
        gamma = 1 + rng.uniform(0.05, 1.0)
        b = mrt.b_from_gamma(gamma)
        state = (rng.uniform(0.1, 10), rng.uniform(-3, 3), rng.uniform(-3, 3), rng.uniform(0.1, 2))
        f = np.asarray(mrt.feq(*state, b), dtype=np.float64)
        yield "equilibrium", f.astype(np.float32)
        yield "perturbed", (f * (1 + 1e-3 * rng.standard_normal(16))).astype(np.float32)
        # signs and magnitudes over nine decades
        yield "wide", (rng.choice([-1.0, 1.0], 16) * 10.0 ** rng.uniform(-6, 3, 16)).astype(np.float32)
        # opposite populations nearly equal: the momenta cancel
        c = rng.uniform(0.1, 1, 16)
        c[2::4] = c[0::4] * (1 + 1e-6 * rng.standard_normal(4))
        c[3::4] = c[1::4] * (1 + 1e-6 * rng.standard_normal(4))
        yield "cancelling", c.astype(np.float32)


def test_fp32_conserved_sums_are_correctly_rounded():
    """The all-FP32 form's compensated conserved moments against exact
    rational sums of the same FP32 terms: within one unit in the last place
    always (the error-free transformations' bound) and the correctly rounded
    value in nearly every case, on equilibria, perturbed equilibria,
    cancelling momenta and terms over nine decades.  Plain FP32 sums of the
    same terms miss the correctly rounded value often, so the bound is a
    test of the compensation."""
    rng = np.random.default_rng(11)
    M = mrt.transformation_matrix()
    M32 = M[:4].astype(np.float32)
    hits = plain_hits = total = 0
    for kind, f in _fp32_cases(rng, 300):
        got = lib.host_conserved_fp32(f)
        plain = np.zeros(4, dtype=np.float32)
        for i in range(16):
            plain = plain + M32[:, i] * f[i]
        for r, ex in enumerate(_fp32_conserved_exact(f)):
            rounded = np.float32(float(ex))
            ulp = float(np.spacing(np.abs(rounded)))
            assert abs(float(got[r]) - float(ex)) <= ulp, (kind, r, got[r], float(ex))
            hits += got[r] == rounded
            plain_hits += plain[r] == rounded
            total += 1
    print("correctly rounded:", hits, "of", total, "; plain FP32 sums:", plain_hits)
    assert hits >= 0.999 * total
    assert plain_hits < 0.9 * total
