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


def test_rm_instability_layout():
    """Section (d): 360 x 100 cells on 0.36 x 0.1, the three printed states,
    the interface x = 0.24 + 0.005 sin(pi/2 + 40 pi y) (period 0.05 = 50
    rows), inflow right, reflecting left, periodic top and bottom."""
    c = W.rm_instability()
    assert (c.nx, c.ny) == (360, 100) and c.dx == pytest.approx(0.001) and c.dy == pytest.approx(0.001)
    assert c.bc == ("reflect", "eq", "periodic", "periodic")
    _, rh = _golden()
    mach, rho1, p1, rho2, u2, p2, tol = rh[0]
    shocked = W.RM_STATES["shocked"]
    assert shocked == (rho2, u2, 0.0, p2)
    assert W.RM_STATES["heavy"] == (rho1, 0.0, 0.0, p1)
    assert c.side_state[1] == pytest.approx((rho2, u2, 0.0, p2 / rho2), rel=1e-15)
    # far-field states: light gas at the left wall, shocked gas at the inflow
    assert c.rho[:, 0] == pytest.approx(0.1358) and c.T[:, 0] == pytest.approx(1 / 0.1358)
    assert c.rho[:, -1] == pytest.approx(rho2) and c.ux[:, -1] == pytest.approx(u2)
    # heavy gas between interface and shock (widest at the troughs, row 25:
    # interface 0.235, shock 0.25), at rest, p = 1
    k = 242
    # (the two 2-cell ramps overlap slightly there: within 1 %)
    assert c.rho[25, k] == pytest.approx(1.0, rel=1e-2)
    assert c.rho[25, k] * c.T[25, k] == pytest.approx(1.0, rel=1e-2)
    assert abs(c.ux[25, k]) < 1e-2 * abs(u2)
    # the interface (rho = (0.1358 + 1) / 2; linear interpolation between cell
    # centres, within 0.15 cells) sits at 0.245 on rows y = 0.0005 and
    # at 0.235 half a period later, and the field repeats every 50 rows
    def crossing(row):
        r = c.rho[row]
        k = int(np.argmax(r > 0.5 * (0.1358 + 1.0)))
        return (k - 0.5 + (0.5679 - r[k - 1]) / (r[k] - r[k - 1])) * c.dx
    y0 = 0.5 * c.dy
    assert crossing(0) == pytest.approx(0.24 + 0.005 * np.cos(40 * np.pi * y0), abs=1.5e-4)
    assert crossing(25) == pytest.approx(0.24 + 0.005 * np.cos(40 * np.pi * (25.5 * c.dy)), abs=1.5e-4)
    assert np.allclose(c.rho[:50], c.rho[50:], rtol=1e-12, atol=0)
    assert c.s[4] == 2e3 and np.all(c.s[5:] == 1e5) and np.all(c.s[:4] == 0) and c.dt == 1e-5


def test_strong_shock_tube_states_and_rates():
    """Section (b): printed states and parameters; MRT rates s_5 = 5e3,
    s_6 = 1e4, others 1e5; SRT tau = 1e-5 (all rates 1e5); the pressures
    rho T are Toro's test-5 values."""
    m = W.strong_shock_tube(1.4, srt=False, ny=1)
    s = W.strong_shock_tube(5 / 3, srt=True, ny=1)
    assert m.dx == 0.002 and m.dt == 1e-6 and m.nsteps == 130000
    assert m.s[4] == 5e3 and m.s[5] == m.s[6] == 1e4 and np.all(m.s[7:] == 1e5)
    assert np.allclose(s.s[4:], 1e5, rtol=1e-15) and np.all(s.s[:4] == 0)
    L, R = W.STRONG_SHOCK_LEFT, W.STRONG_SHOCK_RIGHT
    assert L[0] * L[3] == pytest.approx(460.894, rel=2e-6)
    assert R[0] * R[3] == pytest.approx(46.0950, rel=2e-6)
    x0 = m.meta["x0"]
    xc = (np.arange(m.nx) + 0.5) * m.dx
    assert np.all(m.rho[0][xc < x0] == L[0]) and np.all(m.rho[0][xc > x0] == R[0])
    assert m.bc == ("eq", "eq", "periodic", "periodic")


def test_one_row_oracle_equals_full_tube_oracle():
    """The shock tubes are uniform in y and periodic in y: the oracle on one
    row reproduces every row of the four-row oracle bit for bit (the batch
    parity test relies on this to run the long tubes' oracle cheaply)."""
    from helpers import one_row, oracle_run
    c = W.tube_batch(3, seed=5, nx_range=(60, 90), nsteps=60)[2]
    full, _ = oracle_run(c, 60)
    row, _ = oracle_run(one_row(c), 60)
    for j in range(c.ny):
        assert np.array_equal(full[:, j], row[:, 0])


def test_paper_riemann2d_layout():
    """Section (c): quadrant i holds the printed state i (1 upper right,
    counted anticlockwise), sharp interfaces through the centre, the printed
    rates and time step on the printed 0.002 grid."""
    c = W.paper_riemann2d()
    assert (c.nx, c.ny, c.dx, c.dy, c.dt, c.nsteps) == (500, 500, 0.002, 0.002, 1e-5, 12000)
    corners = {(-1, -1): 0, (-1, 0): 1, (0, 0): 2, (0, -1): 3}   # (row, col) -> quadrant index
    for (j, i), q in corners.items():
        got = (c.rho[j, i], c.ux[j, i], c.uy[j, i], c.T[j, i])
        assert np.allclose(got, W.PAPER_QUADRANTS[q]), (q, got)
    assert set(np.unique(c.rho)) == {s[0] for s in W.PAPER_QUADRANTS}
    assert c.s[7] == c.s[8] == 2e4 and np.all(np.delete(c.s[4:], [3, 4]) == 3e3)
    srt = W.paper_riemann2d(srt=True, srt_rate=2e4)
    assert np.all(srt.s[4:] == 2e4) and np.all(srt.s[:4] == 0)
