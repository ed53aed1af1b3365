"""Linear stability of the paper's strong-shock configuration (section (b))
under the library's reading of the discretisation (unsplit forward Euler,
per-axis Lax-Wendroff), from the oracle's amplification spectrum.  It
explains which runs of that section survive the paper's 130,000 steps."""
import numpy as np
import pytest

from oracle import mrt, stability
from paper_1004_5442_amd import workloads as W


def _amp(gamma, srt, state, reading="unsplit", n_theta=65):
    c = W.strong_shock_tube(gamma, srt, ny=1)
    p = mrt.Params(gamma=gamma, s=c.s, dt=c.dt, dx=c.dx, dy=c.dy)
    return stability.max_amplification(state, p, n_theta=n_theta, one_d=True, reading=reading)


def test_gamma_7_5_runs_are_stable_in_1d():
    for srt in (False, True):
        for st in (W.STRONG_SHOCK_LEFT, W.STRONG_SHOCK_RIGHT):
            assert _amp(1.4, srt, st) <= 1.0 + 1e-8


def test_gamma_5_3_mrt_is_unstable_at_the_hot_state():
    g = _amp(5.0 / 3.0, False, W.STRONG_SHOCK_LEFT)
    assert 1.0 + 1e-4 < g < 1.0 + 1e-3
    # SRT at the same state grows 10x slower
    assert _amp(5.0 / 3.0, True, W.STRONG_SHOCK_LEFT) < 1.0 + 5e-5


def test_2d_modes_destabilise_the_mrt_tube():
    """With more than one row a y-wave (theta_y = pi/2, what a 4-row periodic
    tube carries) is unstable even at gamma = 7/5: the 1D problem is run on
    one row."""
    c = W.strong_shock_tube(1.4, False, ny=4)
    p = mrt.Params(gamma=1.4, s=c.s, dt=c.dt, dx=c.dx, dy=c.dy)
    worst = max(float(np.max(np.abs(stability.mode_rates(W.STRONG_SHOCK_LEFT, p, tx, np.pi / 2))))
                for tx in np.linspace(-np.pi, np.pi, 65))
    assert worst > 1.0 + 1e-4


# growth per step of the gamma = 5/3 MRT run at the hot left state under each
# reading (97 phase angles), as printed in the design notes
READING_GROWTH_5_3 = {"unsplit": 2.05e-4, "split": 1.46e-4, "rhs_taylor": 1.82e-4,
                      "trapezoid": 1.80e-4, "exp_collision": 1.81e-4}


def test_no_reading_of_the_discretisation_passage_stabilises_gamma_5_3():
    """Section (b) reports the gamma = 5/3 MRT run of the strong-shock
    problem as successful.  Every reading of the time/space passage the
    stability tool forms (forward Euler unsplit or split either way round,
    Lax-Wendroff's Taylor term on the whole right-hand side collision
    included, a Crank-Nicolson or an exact collision) keeps gamma = 7/5 stable
    at both states and leaves the hot left state of gamma = 5/3 growing by
    1.5-2.1e-4 per step (e^19 to e^27 over the 130,000 steps)."""
    for reading in stability.READINGS:
        for st in (W.STRONG_SHOCK_LEFT, W.STRONG_SHOCK_RIGHT):
            assert _amp(1.4, False, st, reading, 97) <= 1.0 + 1e-7, reading
        g = _amp(5.0 / 3.0, False, W.STRONG_SHOCK_LEFT, reading, 97)
        assert g - 1.0 == pytest.approx(READING_GROWTH_5_3[reading], rel=0.02), (reading, g)


def test_hot_state_is_unstable_before_discretisation():
    """Why no reading helps: the model itself, continuous in time and space
    (eigenvalues of -i k v_x - J_C), has modes growing at grid-scale
    wavenumbers at the hot left state, ~1e4 per unit time at k dx = pi for
    either gamma (equilibria with negative populations make the linearised
    collision not dissipative there).  Only the Lax-Wendroff damping,
    c^2 (1 - cos theta) per step at Courant numbers of at most 3e-3, holds
    them down, and at gamma = 5/3 it falls short; at the cold right state the
    continuous model is stable for gamma = 7/5."""
    for gamma in (1.4, 5.0 / 3.0):
        c = W.strong_shock_tube(gamma, False, ny=1)
        p = mrt.Params(gamma=gamma, s=c.s, dt=c.dt, dx=c.dx, dy=c.dy)
        assert stability.semi_discrete_growth(W.STRONG_SHOCK_LEFT, p, np.pi) > 5e3
    c = W.strong_shock_tube(1.4, False, ny=1)
    p = mrt.Params(gamma=1.4, s=c.s, dt=c.dt, dx=c.dx, dy=c.dy)
    worst = max(stability.semi_discrete_growth(W.STRONG_SHOCK_RIGHT, p, th)
                for th in np.linspace(0.01, np.pi, 64))
    assert worst < 1e-6


def test_paper_riemann2d_quadrant_growth_rates():
    """Linear stability of the four printed quadrant states of section (c)
    at the paper's parameters (dx = 0.002, dt = 1e-5; MRT s_8 = s_9 = 2e4,
    other rates 3e3): quadrant 1 is stable, quadrants 2 and 4 grow by
    ~4.9e-4 per step and the cold supersonic quadrant 3 (T = 0.21, Mach 3.14)
    by ~1.55e-3: e^18.6 over the 12,000 steps.  Rounding seeds that mode: FP64
    rounding (1e-16) stays far below O(1) (~1e-8) while FP32 storage rounding
    (6e-8) reaches it, which is why the FP64 run reaches t = 0.12 and the
    FP32-storage run breaks down near step 11,500."""
    c = W.paper_riemann2d(n=50)
    p = mrt.Params(gamma=1.4, s=c.s, dt=1e-5, dx=0.002, dy=0.002)
    g = [stability.max_amplification(st, p, n_theta=33) - 1.0 for st in W.PAPER_QUADRANTS]
    assert g[0] < 1e-12
    assert g[1] == pytest.approx(4.87e-4, rel=0.05) and g[3] == pytest.approx(g[1], rel=1e-6)
    assert g[2] == pytest.approx(1.55e-3, rel=0.05)
    growth = np.exp(g[2] * 12000)
    assert 1e-16 * growth < 1e-6 < 6e-8 * growth


def test_sod_with_the_paper_shock_tube_rates_breaks_down():
    """Why the Sod configuration does not use the paper's strong-shock rates:
    with s_5 = 5e3, s_6 = 1e4 (section (b)) on the 400-cell Sod tube at
    dt = 1e-5 the oracle turns non-physical (T < 0 at the contact) after ~330
    steps, short of the configured 1000; with the rates the Sod workload uses
    (s_5 = 500, s_6 = 1e3: ten times the viscosity, the paper having run at
    T = 8-77 where its rates give that much more) it stays physical."""
    import dataclasses

    from helpers import one_row, oracle_params
    base = one_row(W.sod_tube())

    def first_bad_step(s, nsteps=1000):
        c = dataclasses.replace(base, s=s)
        p = oracle_params(c)
        f = mrt.init_populations(c.rho, c.ux, c.uy, c.T, p)
        for n in range(1, nsteps + 1):
            f = mrt.step(f, p)
            rho, _, _, T = mrt.macroscopic(f, p.b)
            if not (np.isfinite(f).all() and rho.min() > 0 and T.min() > 0):
                return n
        return None

    bad = first_bad_step(W.rates(5e3, 1e4, 0.71, 1e5))
    assert bad is not None and 200 < bad < 500, bad
    assert first_bad_step(base.s) is None
