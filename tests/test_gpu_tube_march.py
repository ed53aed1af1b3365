"""GPU parity of the tube march: four time steps per pass for tubes of 1, 2
or 4 periodic rows with fixed-equilibrium x sides (the shock tubes of
section (b)), batched or single, each block holding all rows of a tube in
registers and storing 248 of the 256 columns it computes.  Against the FP64
oracle and against the same grids advanced one step per pass."""
import dataclasses

import numpy as np
import pytest

from helpers import field_errors, fp32_tolerances, fp64_rounding_spread, one_row, oracle_run
from oracle import mrt
from paper_1004_5442_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd.batch import Batch  # noqa: E402
from paper_1004_5442_amd.lib import MRTError, UnstableError  # noqa: E402
from paper_1004_5442_amd.solver import solver_for_case  # noqa: E402

TUBE_WIDTH = 248      # columns one block stores (256 less one per step on either side)


def _tubes(sizes, seed=0, ny=4):
    """Shock tubes of the given lengths: one block and its edges (1, 3,
    247, 248, 249), two and three blocks with ragged ends."""
    out = []
    for k, nx in enumerate(sizes):
        c = W.tube_batch(1, seed=seed + k, nx_range=(nx, nx), ny=ny)[0]
        out.append(dataclasses.replace(c, name=f"tube_nx{nx}_ny{ny}"))
    return out


SIZES = [1, 3, 200, TUBE_WIDTH - 1, TUBE_WIDTH, TUBE_WIDTH + 1, 2 * TUBE_WIDTH,
         2 * TUBE_WIDTH + 1, 745]


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp32"])
def test_tube_march_matches_oracle_and_single_steps(precision):
    """13 steps per call over three calls (three four-step passes and one
    single step each) on tubes of one to three blocks: every tube against
    the FP64 oracle (the stated 1e-5 per field, or twice the FP32-storage
    error) and against the same batch one step per pass.  The pure FP32
    form equals it bit for bit (the same per-cell arithmetic, its FP32
    transforms fused the same way everywhere); with the FP64 collision the
    compiler may fuse the FP64 arithmetic differently in the two kernels, so
    the bound is two FP32 ulps of the population scale."""
    cases = _tubes(SIZES)
    one = Batch(cases, precision)
    one.set_steps_per_pass(1)             # the batch of tubes defaults to the tube march
    tube = Batch(cases, precision)
    assert tube.steps_per_pass() == (4, 4)
    tube.set_steps_per_pass(4)
    assert tube.steps_per_pass() == (4, 4)
    for call in range(3):
        print(f"call {call} {precision}", flush=True)
        one.step(13)
        tube.step(13)
    for i, c in enumerate(cases):
        want, p = oracle_run(c, 39)
        err = field_errors(tube.moments(i), mrt.macroscopic(want, p.b))
        tol = fp32_tolerances(c, 39, want)
        a, b = tube.populations(i), one.populations(i)
        d = float(np.max(np.abs(a - b)) / np.abs(b).max())
        print(c.name, err, "vs one step per pass", d, flush=True)
        assert all(err[k] < tol[k] for k in err), (c.name, err, tol)
        if precision == "fp32":
            assert d == 0.0, (c.name, d)
        else:
            assert d <= 2.4e-7, (c.name, d)


def test_tube_march_across_graph_replays_and_step_counts():
    """Step counts that exercise the captured passes (64 passes per graph
    replay) and every remainder of single steps (1 to 3), against one step
    per pass."""
    cases = _tubes([300, 600], seed=5)
    one = Batch(cases, "fp32")
    one.set_steps_per_pass(1)
    tube = Batch(cases, "fp32")
    tube.set_steps_per_pass(4)
    for n in (1, 2, 3, 4, 7, 258):
        print(f"{n} steps", flush=True)
        one.step(n)
        tube.step(n)
        for i in range(len(cases)):
            assert np.array_equal(tube.populations(i), one.populations(i)), (n, i)


@pytest.mark.parametrize("ny", [1, 2, 4])
def test_tube_march_fp64_matches_oracle_and_single_steps(ny):
    """FP64 storage, tubes of one, two and four rows (one to three blocks),
    13 steps per call over three calls: against the oracle at 1e-12 of the
    population scale and against one step per pass to rounding order
    (1e-13: the FP64 collision may fuse products into FMAs differently in
    the two kernels)."""
    cases = _tubes([3, TUBE_WIDTH, TUBE_WIDTH + 1, 600], seed=7, ny=ny)
    one = Batch(cases, "fp64")
    one.set_steps_per_pass(1)
    tube = Batch(cases, "fp64")
    tube.set_steps_per_pass(4)
    assert tube.steps_per_pass() == (4, ny)
    for call in range(3):
        print(f"call {call} fp64 ny {ny}", flush=True)
        one.step(13)
        tube.step(13)
    for i, c in enumerate(cases):
        want, p = oracle_run(c, 39)
        got = tube.populations(i)
        err = float(np.max(np.abs(got - want)) / np.abs(want).max())
        d = float(np.max(np.abs(got - one.populations(i))) / np.abs(want).max())
        print(c.name, "vs oracle", err, "vs one step per pass", d, flush=True)
        assert err <= 1e-12, (c.name, err)
        assert d <= 1e-13, (c.name, d)


@pytest.mark.parametrize("ny", [1, 2])
def test_tube_march_one_and_two_rows_fp32(ny):
    """Tubes of one and two periodic rows in FP32 storage with FP64
    collision: against the oracle (the stated 1e-5 or twice the
    FP32-storage error) and against one step per pass (two FP32 ulps)."""
    cases = _tubes([200, TUBE_WIDTH + 1, 745], seed=4, ny=ny)
    one = Batch(cases, "fp32_eq64")
    one.set_steps_per_pass(1)
    tube = Batch(cases, "fp32_eq64")
    tube.set_steps_per_pass(4)
    one.step(41)
    tube.step(41)
    for i, c in enumerate(cases):
        want, p = oracle_run(c, 41)
        err = field_errors(tube.moments(i), mrt.macroscopic(want, p.b))
        tol = fp32_tolerances(c, 41, want)
        a, b = tube.populations(i), one.populations(i)
        d = float(np.max(np.abs(a - b)) / np.abs(b).max())
        print(c.name, err, "vs one step per pass", d, flush=True)
        assert all(err[k] < tol[k] for k in err), (c.name, err, tol)
        assert d <= 2.4e-7, (c.name, d)


def test_tube_march_rejected_outside_its_cover():
    """Instances of other heights, mixed heights in one batch, or
    non-equilibrium x sides: four steps per pass are refused (batch and
    single grid); a 2D grid too."""
    tubes = _tubes([300])
    eight = W.tube_batch(1, seed=1, nx_range=(300, 300), ny=8)[0]
    with pytest.raises(MRTError):
        Batch(tubes + [eight], "fp32_eq64").set_steps_per_pass(4)
    two = _tubes([300], ny=2)
    with pytest.raises(MRTError):
        Batch(tubes + two, "fp64").set_steps_per_pass(4)
    outflow = dataclasses.replace(tubes[0], bc=("eq", "outflow", "periodic", "periodic"))
    with pytest.raises(MRTError):
        Batch([outflow], "fp32_eq64").set_steps_per_pass(4)
    with pytest.raises(MRTError):
        Batch(tubes, "fp32_eq64").set_steps_per_pass(3)
    s = solver_for_case(eight, "fp64")
    with pytest.raises(MRTError):
        s.set_steps_per_pass(4)
    s.close()
    s = solver_for_case(W.riemann2d(n=64, seed=0), "fp32_eq64")
    with pytest.raises(MRTError):
        s.set_steps_per_pass(4)
    s.close()


def test_single_grid_sod_tube_fp64_by_the_tube_march():
    """The plain method's Sod tube (400 x 4, FP64, fixed ends, periodic in
    y) on a single grid, 1000 steps by the tube march: the fields against
    the oracle at 1e-12, as with one step per pass."""
    case = W.sod_tube()
    want, p = oracle_run(case, case.nsteps)
    s = solver_for_case(case, "fp64")
    s.set_steps_per_pass(4)
    assert s.steps_per_pass() == (4, 4)
    s.step(case.nsteps)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    s.close()
    print("sod fp64 tube march", err, flush=True)
    assert max(err.values()) < 1e-12, err


def test_single_grid_strong_shock_tube_by_the_tube_march():
    """The paper's strong-shock tube (gamma 7/5, 1100 x 1, FP64, fixed
    ends), 2002 steps by the tube march (500 passes and two single steps):
    against the oracle within 1e-12 or four times the oracle's own spread
    under one-ulp perturbations (the hot supersonic states amplify
    rounding), the bound of the one-step test of the same case."""
    case = W.strong_shock_tube(1.4, False, ny=1)
    want, p = oracle_run(case, 2002)
    s = solver_for_case(case, "fp64")
    s.set_steps_per_pass(4)
    s.step(2002)
    got = s.populations()
    s.close()
    err = float(np.max(np.abs(got - want)) / np.abs(want).max())
    tol = max(1e-12, 4.0 * fp64_rounding_spread(case, 2002, want))
    print("strong shock tube march", err, "tolerance", tol, flush=True)
    assert err <= tol


def test_tube_march_reports_unhealthy_cells():
    """A tube stepped far past its stability limit (dt 10^5 times larger,
    rates scaled to keep s dt) goes negative at its diaphragm within the
    first four-step pass: the health flag reports it, and the flag is
    cleared by the report."""
    cases = _tubes([300, 300], seed=2)
    c = cases[1]
    bad = dataclasses.replace(c, dt=0.5, s=list(np.asarray(c.s) * (c.dt / 0.5)))
    b = Batch([cases[0], bad], "fp32_eq64")
    b.set_steps_per_pass(4)
    b.step(4)
    with pytest.raises(UnstableError):
        b.moments(0)
    good = Batch(cases, "fp32_eq64")
    good.set_steps_per_pass(4)
    good.step(8)
    good.moments(0)


_FULL = {}


def _full_tube_march():
    if not _FULL:
        cases = W.tube_batch(512, seed=0)
        b = Batch(cases, "fp32_eq64")
        b.set_steps_per_pass(4)
        b.step(1000)
        r = [c.meta["pressure_ratio"] for c in cases]
        g = [c.gamma for c in cases]
        sel = {"max_pressure_ratio": int(np.argmax(r)), "min_gamma": int(np.argmin(g)),
               "max_gamma": int(np.argmax(g)), "longest": int(np.argmax([c.nx for c in cases]))}
        _FULL["cases"] = cases
        _FULL["sel"] = sel
        _FULL["moments"] = {i: b.moments(i) for i in set(sel.values())}
        b.close()
    return _FULL


@pytest.mark.parametrize("which", ["max_pressure_ratio", "min_gamma", "max_gamma", "longest"])
def test_full_batch_512_tubes_tube_march(which):
    """The 512-tube batch, 1000 steps by the tube march, FP32 storage with
    FP64 collision: the selected tube's rho, u, T against the FP64 oracle
    (run on one row), to the stated 1e-5 or twice the FP32-storage error."""
    full = _full_tube_march()
    i = full["sel"][which]
    c = full["cases"][i]
    c1 = one_row(c)
    want, p = oracle_run(c1, 1000)
    got = [a[:1] for a in full["moments"][i]]
    err = field_errors(got, mrt.macroscopic(want, p.b))
    tol = fp32_tolerances(c1, 1000, want)
    print(which, c.name, f"nx {c.nx}", "err", err, "tol", tol, flush=True)
    assert all(err[k] < tol[k] for k in err), (c.name, err, tol)


def test_tube_march_prepared_graphs_and_autotuned_single_grid():
    """Graphs captured ahead of the steps (prepare, as the benchmark does)
    replay the same passes as graphs captured on first use (bit for bit);
    and the single-grid autotuner, which times the tube march on a tube,
    leaves a launch whose steps equal single steps to rounding order (on
    the paper's strong-shock tube, whose hot supersonic states amplify
    rounding: 1e-12 or four times the oracle's own one-ulp spread)."""
    cases = _tubes([300, 700], seed=8)
    a, b = Batch(cases, "fp32_eq64"), Batch(cases, "fp32_eq64")
    a.set_steps_per_pass(4)
    b.set_steps_per_pass(4)
    a.prepare(258)
    a.step(258)
    b.step(258)
    for i in range(len(cases)):
        assert np.array_equal(a.populations(i), b.populations(i)), i
    case = W.strong_shock_tube(1.4, False, ny=1)
    tuned = solver_for_case(case, "fp64")
    tuned.autotune(4)
    print("autotuned", tuned.steps_per_pass(), tuned.tile(), flush=True)
    one = solver_for_case(case, "fp64")
    one.set_steps_per_pass(1, 0)
    tuned.step(202)
    one.step(202)
    got, ref = tuned.populations(), one.populations()
    d = float(np.max(np.abs(got - ref)) / np.abs(ref).max())
    want, _ = oracle_run(case, 202)
    tol = max(1e-12, 4.0 * fp64_rounding_spread(case, 202, want))
    print("autotuned against single steps", d, "tolerance", tol, flush=True)
    assert d <= tol
    tuned.close()
    one.close()
