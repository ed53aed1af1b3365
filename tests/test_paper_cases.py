"""Linear stability of the paper's strong-shock configuration (section (b))
under the library's reading of the discretisation (unsplit forward Euler,
per-axis Lax-Wendroff), from the oracle's amplification spectrum.  It
explains which runs of that section survive the paper's 130,000 steps."""
import numpy as np

from oracle import mrt, stability
from paper_1004_5442_amd import workloads as W


def _amp(gamma, srt, state):
    c = W.strong_shock_tube(gamma, srt, ny=1)
    p = mrt.Params(gamma=gamma, s=c.s, dt=c.dt, dx=c.dx, dy=c.dy)
    return stability.max_amplification(state, p, n_theta=65, one_d=True)


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
