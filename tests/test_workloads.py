"""Seeded input generators: reproducible, and pinned to the numbers the
paper prints for its initial states."""
import os

import numpy as np
import pytest

from paper_1004_5442_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_printed_states.txt")


def _golden():
    quads, rh = [], []
    with open(GOLDEN) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            tok = line.split()
            if tok[0] == "RH":
                rh.append([float(t) for t in tok[1:]])
            else:
                quads.append([float(t) for t in tok])
    return quads, rh


def test_paper_quadrant_mach_numbers():
    quads, _ = _golden()
    for q, rho, u1, u2, Tnum, mach, tol in quads:
        st = W.PAPER_QUADRANTS[int(q) - 1]
        assert st[0] == rho and st[1] == u1 and st[2] == u2
        assert st[3] == pytest.approx(Tnum / rho, rel=1e-15)
        got = np.hypot(st[1], st[2]) / np.sqrt(1.4 * st[3])
        assert got == pytest.approx(mach, rel=tol)


def test_rankine_hugoniot_reproduces_paper_rm_state():
    _, rh = _golden()
    mach, rho1, p1, rho2, u2, p2, tol = rh[0]
    post = W.rankine_hugoniot(mach, (rho1, 0.0, 0.0, p1 / rho1), 1.4, direction=-1)
    assert post[0] == pytest.approx(rho2, rel=tol)
    assert post[1] == pytest.approx(u2, rel=tol)
    assert post[0] * post[3] == pytest.approx(p2, rel=tol)


def test_generators_are_seeded_and_in_range():
    a = W.quadrant_states(5)
    assert a == W.quadrant_states(5)
    assert a != W.quadrant_states(6)
    for rho, ux, uy, T in a:
        assert 0.5 <= rho <= 1.5 and 0.1 <= rho * T <= 1.5
        assert np.hypot(ux, uy) <= 1.5 * np.sqrt(1.4 * T) + 1e-12
    tubes = W.tube_batch(64, seed=1)
    assert [t.nx for t in tubes] == [t.nx for t in W.tube_batch(64, seed=1)]
    for t in tubes:
        assert 200 <= t.nx <= 4000 and t.ny == 4
        assert 1.1 <= t.gamma <= 1.67 and 0.5 <= t.Pr <= 2.0
        assert 2.0 <= t.meta["pressure_ratio"] <= 1000.0
        assert np.all(t.s[4:] * t.dt <= 1.0 + 1e-12)


def test_smooth_noise_is_periodic_unit_std():
    n = W.smooth_noise(64, 0)
    assert n.std() == pytest.approx(1.0) and abs(n.mean()) < 1e-12
    # smoothing over 8 cells: neighbouring cells are strongly correlated,
    # across the periodic seam as much as inside
    c_in = np.corrcoef(n[:, 10], n[:, 11])[0, 1]
    c_seam = np.corrcoef(n[:, -1], n[:, 0])[0, 1]
    assert c_in > 0.95 and c_seam > 0.95


def test_shock_bubble_layout():
    c = W.shock_bubble(n=256, ny=256)
    assert c.bc == ("eq", "outflow", "reflect", "reflect")
    post = c.meta["post"]
    assert post[0] == pytest.approx(5.0) and post[0] * post[3] == pytest.approx(29 * 0.6)
    assert c.rho[128, 2] == pytest.approx(post[0], rel=1e-6)
    assert c.rho[128, 64] == pytest.approx(3.0, rel=1e-6)      # bubble centre (0.25, 0.5)
    assert c.rho[128, 200] == pytest.approx(1.0, rel=1e-6)
