"""Pins of the exact Riemann solver used to validate shock tubes."""
import math
import os

import numpy as np
import pytest

from oracle import riemann

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "toro_star_states.txt")


def _rows():
    out = []
    with open(GOLDEN) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                out.append([float(v) for v in line.split()])
    return out


@pytest.mark.parametrize("row", _rows())
def test_textbook_star_states(row):
    rl, ul, pl, rr, ur, pr, ps, us, tol = row
    p, u = riemann.star_state((rl, ul, pl), (rr, ur, pr), 1.4)
    assert p == pytest.approx(ps, rel=tol)
    assert u == pytest.approx(us, abs=tol * max(1.0, abs(us)))


@pytest.mark.parametrize("gamma", [1.1, 1.4, 5.0 / 3.0])
def test_shock_satisfies_rankine_hugoniot(gamma):
    left, right = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    xi = np.linspace(-3, 3, 6001)
    rho, u, p = riemann.sample(left, right, gamma, xi)
    # right-moving shock: find the jump from the pre-shock state
    i = np.where(np.abs(rho - right[0]) > 1e-12)[0].max()
    r1, u1, p1 = rho[i + 1], u[i + 1], p[i + 1]
    r2, u2, p2 = rho[i], u[i], p[i]
    S = (r2 * u2 - r1 * u1) / (r2 - r1)          # mass conservation fixes the speed
    # momentum and energy fluxes in the shock frame are continuous
    m = r1 * (u1 - S)
    assert m * (u2 - S) + p2 == pytest.approx(m * (u1 - S) + p1, rel=1e-12)
    h = lambda r, pp, w: gamma / (gamma - 1) * pp / r + 0.5 * w * w
    assert h(r2, p2, u2 - S) == pytest.approx(h(r1, p1, u1 - S), rel=1e-12)


def test_rarefaction_is_isentropic_and_symmetric_case():
    gamma = 1.4
    left, right = (1.0, -1.0, 0.5), (1.0, 1.0, 0.5)
    p, u = riemann.star_state(left, right, gamma)
    assert u == pytest.approx(0.0, abs=1e-14)
    xi = np.linspace(-3, 3, 601)
    rho, uu, pp = riemann.sample(left, right, gamma, xi)
    np.testing.assert_allclose(pp / rho ** gamma, 0.5, rtol=1e-12)
    np.testing.assert_allclose(uu, -uu[::-1], atol=1e-13)
