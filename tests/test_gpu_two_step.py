"""GPU parity of the two-steps-per-pass kernel (mrt_set_steps_per_pass).

One launch advances the state two steps: f^{n+1} lives only in registers
(FP32, as the single-step kernel would store it), recomputed on the two halo
rows of each band and on the two halo columns of each block, with the
boundary rules applied to it in the kernel.  Against the FP64 oracle (the
stated 1e-5 on rho, u, T) and against the single-step kernel on the same
input (which rounds f^{n+1} to FP32 the same way: agreement to a few FP32
ulps), on ragged shapes, every boundary kind on every side, band heights
from 1 to 32 rows, odd step counts (a single step ends the run), graph
replays, and the 4096^2 shock-bubble grid at the benchmark's configuration.
"""
import numpy as np
import pytest

from helpers import field_errors, oracle_params, oracle_run, smooth_case
from oracle import mrt
from paper_1004_5442_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd.solver import Solver, solver_for_case  # noqa: E402

BC_SETS = [
    ("periodic", "periodic", "periodic", "periodic"),
    ("reflect", "reflect", "reflect", "reflect"),
    ("eq", "outflow", "reflect", "reflect"),
    ("reflect", "eq", "periodic", "periodic"),
    ("outflow", "reflect", "eq", "outflow"),
    ("periodic", "periodic", "reflect", "eq"),
]
# (257, 4) and (1, 4) with 4-row bands: where both y sides are periodic the
# band is a whole periodic height of four rows, and the kernel takes f^{n+1}
# of its last two rows from the wrapped rows it computed first
SHAPES = [((150, 37), 8), ((64, 5), 2), ((1, 7), 3), ((65, 1), 1), ((256, 12), 5),
          ((257, 9), 32), ((512, 3), 1), ((300, 40), 32), ((2, 2), 1), ((257, 4), 4),
          ((1, 4), 4)]


def close_to_single_step(a, b):
    """populations of the two paths: equal up to a few FP32 roundings"""
    scale = np.abs(b).max()
    return float(np.max(np.abs(a - b)) / scale)


@pytest.mark.parametrize("bc", BC_SETS)
@pytest.mark.parametrize("shape,rows", SHAPES)
def test_two_step_matches_oracle_and_single_step(bc, shape, rows):
    nx, ny = shape
    nsteps = 13                     # six two-step passes and one single step
    case = smooth_case(nx, ny, bc, seed=3 * nx + ny)
    print(f"case {case.name} bc={bc} rows={rows} fp32_eq64 two-step", flush=True)
    want, p = oracle_run(case, nsteps)
    one = solver_for_case(case, "fp32_eq64")
    one.set_steps_per_pass(1, 0)
    one.step(nsteps)
    two = solver_for_case(case, "fp32_eq64")
    two.set_steps_per_pass(2, rows)
    two.step(nsteps)
    err = field_errors(two.moments(), mrt.macroscopic(want, p.b))
    d = close_to_single_step(two.populations(), one.populations())
    print("vs oracle", err, "vs single step", d, flush=True)
    assert max(err.values()) < 1e-5, err
    assert d < 1e-6, d
    one.close()
    two.close()


@pytest.mark.parametrize("bc", BC_SETS)
@pytest.mark.parametrize("shape,rows", SHAPES)
def test_fp64_two_step_matches_oracle_and_single_step(bc, shape, rows):
    """FP64 storage, two steps per pass (one block per CU: both register
    windows in FP64): populations after 13 steps against the oracle at
    1e-12 of their scale, and against the FP64 one-step kernel to rounding
    order (1e-13: the same site arithmetic, f^{n+1} held as the double a
    stored state would be, the FP64 collision's FMA fusion possibly chosen
    differently per unrolled row)."""
    nx, ny = shape
    nsteps = 13
    case = smooth_case(nx, ny, bc, seed=3 * nx + ny)
    print(f"case {case.name} bc={bc} rows={rows} fp64 two-step", flush=True)
    want, p = oracle_run(case, nsteps)
    one = solver_for_case(case, "fp64")
    one.step(nsteps)
    two = solver_for_case(case, "fp64")
    two.set_steps_per_pass(2, rows)
    assert two.steps_per_pass() == (2, min(rows, ny))
    two.step(nsteps)
    got = two.populations()
    err = float(np.max(np.abs(got - want)) / np.abs(want).max())
    d = close_to_single_step(got, one.populations())
    print("vs oracle", err, "vs single step", d, flush=True)
    assert err <= 1e-12, err
    assert d <= 1e-13, d
    one.close()
    two.close()


@pytest.mark.parametrize("rows", [1, 4, 16, 32])
@pytest.mark.parametrize("bc", BC_SETS[1:3])
def test_pure_fp32_form_two_step(bc, rows):
    """Pure FP32 (collision in FP32 with compensated conserved sums): two
    steps per pass against the oracle and against two single steps.  The
    FP32 transforms fuse products into FMAs only within an expression, so
    every row of either march rounds alike and the two paths agree bit for
    bit at every band height."""
    case = smooth_case(300, 40, bc, seed=5)
    print(f"case {case.name} bc={bc} rows={rows} fp32 two-step", flush=True)
    want, p = oracle_run(case, 40)
    one = solver_for_case(case, "fp32")
    one.set_steps_per_pass(1, 0)
    one.step(40)
    s = solver_for_case(case, "fp32")
    s.set_steps_per_pass(2, rows)
    s.step(40)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    d = close_to_single_step(s.populations(), one.populations())
    print("fp32 two-step", err, "vs single step", d, flush=True)
    assert max(err.values()) < 1e-5, err
    assert d == 0.0, d
    s.close()
    one.close()


def test_graph_replays_and_switching_back():
    """Many passes through captured graphs (64-pass chunks plus remainders),
    odd counts, then back to one step per pass (the reflecting ghosts of the
    current state are refreshed by the switch) and forth again."""
    case = smooth_case(300, 40, ("reflect", "eq", "reflect", "outflow"), seed=21)
    print(f"case {case.name} two-step graphs", flush=True)
    total = 0
    s = solver_for_case(case, "fp32_eq64")
    s.set_steps_per_pass(2, 8)
    for n in (129, 2, 7):
        s.step(n)
        total += n
    s.set_steps_per_pass(1, 0)
    s.step(5)
    total += 5
    s.set_steps_per_pass(2, 0)
    s.step(64)
    total += 64
    want, p = oracle_run(case, total)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    print(total, "steps", err, flush=True)
    assert max(err.values()) < 1e-5, err
    s.close()


def test_health_flag_in_two_step_pass():
    from paper_1004_5442_amd.lib import UnstableError
    case = smooth_case(70, 9, BC_SETS[0])
    s = solver_for_case(case, "fp32_eq64")
    s.set_steps_per_pass(2, 0)
    f = s.populations()
    f[:, 4, 33] = np.nan
    s.set_populations(f)
    s.step(2)
    with pytest.raises(UnstableError):
        s.moments()
    s.close()


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp32"])
@pytest.mark.parametrize("row", [0, 3])
def test_health_flag_in_wrapped_four_row_band(precision, row):
    """A NaN in row 0 or row 3 of a 4-row periodic grid stepped in one 4-row
    band (row 3's f^{n+1} is then computed only as the wrapped row -1)."""
    from paper_1004_5442_amd.lib import UnstableError
    case = smooth_case(300, 4, BC_SETS[0], seed=2)
    print(f"case {case.name} {precision} NaN in row {row}", flush=True)
    s = solver_for_case(case, precision)
    s.set_steps_per_pass(2, 4)
    f = s.populations()
    f[:, row, 257] = np.nan
    s.set_populations(f)
    s.step(2)
    with pytest.raises(UnstableError):
        s.moments()
    s.close()


def test_rejected_settings():
    from paper_1004_5442_amd.lib import MRTError
    case = smooth_case(64, 5, BC_SETS[0])
    s = solver_for_case(case, "fp32_eq64")
    for steps, rows in ((3, 0), (0, 0), (2, 65), (2, -1)):
        with pytest.raises(MRTError):
            s.set_steps_per_pass(steps, rows)
    s.set_steps_per_pass(2, 32)                 # accepted: clamped to the 5 rows
    s.step(4)
    s.close()


def test_default_and_autotuned_path():
    """Cache-resident grids default to one step per pass; the autotuner
    times both paths and keeps either, and the state is unchanged by it."""
    case = smooth_case(300, 40, ("reflect", "eq", "periodic", "periodic"), seed=9)
    s = solver_for_case(case, "fp32_eq64")
    assert s.steps_per_pass()[0] == 1
    before = s.populations()
    s.autotune(4)
    assert np.array_equal(s.populations(), before)
    k, rows = s.steps_per_pass()
    print("autotuned", k, rows, s.tile(), flush=True)
    assert k in (1, 2) and rows >= 1
    want, p = oracle_run(case, 9)
    s.step(9)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    assert max(err.values()) < 1e-5, err
    s.close()


def test_default_launch_shapes():
    """The launch a grid gets without autotuning: one step per pass below
    about 1024^2 cells, two from there on (8- or 16-row bands, by storage
    precision), 32 / 64 rows at 4096^2, and the tube march on the shock
    tubes it covers, single or batched."""
    from paper_1004_5442_amd.batch import Batch
    bc = ("outflow",) * 4
    expect = [(768, "fp32_eq64", (1,)), (1024, "fp32_eq64", (2, 8)), (1024, "fp64", (2, 16)),
              (2048, "fp32_eq64", (2, 32)), (2048, "fp64", (2, 64))]
    for n, prec, want in expect:
        s = Solver(n, n, prec, bc)
        got = s.steps_per_pass()
        print(n, prec, got, flush=True)
        assert got[:len(want)] == want, (n, prec, got)
        s.close()
    tube = W.sod_tube()
    s = solver_for_case(tube, "fp32_eq64")
    assert s.steps_per_pass() == (4, 4)
    s.close()
    b = Batch(W.tube_batch(6, seed=2, nx_range=(200, 300)), "fp32_eq64")
    assert b.steps_per_pass() == (4, 4)
    b.close()
    mixed = W.tube_batch(2, seed=2, nx_range=(200, 300)) + [smooth_case(64, 5, bc, seed=1)]
    b = Batch(mixed, "fp32_eq64")
    assert b.steps_per_pass()[0] == 1
    b.close()


@pytest.mark.parametrize("bc", [("reflect", "reflect", "reflect", "reflect"),
                                ("eq", "outflow", "reflect", "reflect")])
def test_autotune_after_two_step_passes(bc):
    """Two-step passes leave the reflecting-wall ghosts of the current
    state stale; the autotuner (which may then choose the one-step kernel,
    whose small-grid form trusts those ghosts) refreshes them first."""
    case = smooth_case(300, 40, bc, seed=17)
    s = solver_for_case(case, "fp32_eq64")
    s.set_steps_per_pass(2, 8)
    s.step(10)
    s.autotune(4)
    print("autotuned", s.steps_per_pass(), s.tile(), flush=True)
    s.step(9)
    want, p = oracle_run(case, 19)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    assert max(err.values()) < 1e-5, err
    s.close()


def test_variants_run_one_step_per_pass():
    """A scheme variant ignores the two-step setting (its own kernels)."""
    case = smooth_case(150, 37, ("eq", "outflow", "reflect", "reflect"), seed=2)
    want, p = oracle_run(case, 6, split=True)
    s = solver_for_case(case, "fp32_eq64")
    s.set_steps_per_pass(2, 0)
    s.set_scheme(split=True)
    s.step(6)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    assert max(err.values()) < 1e-5, err
    s.close()


def test_shock_bubble_4096_two_step_sampled():
    """The benchmark grid (FP32 storage, non-temporal stores; 16-row bands here,
    the default 32 in the sampled test of the full-size module):
    7 steps (three passes and a single step), then patches at the shock, the
    bubble, the walls, inflow, outflow and the corners against the oracle's
    windowed evaluation, and the whole state against the single-step path."""
    from test_gpu_fullsize import compare, shock_bubble_centres
    n, nsteps = 4096, 7
    case = W.shock_bubble(n=n)
    print(f"case {case.name} fp32_eq64 two-step {nsteps} steps", flush=True)
    s = solver_for_case(case, "fp32_eq64")
    assert s.steps_per_pass() == (2, 32)        # the default at this size
    s.set_steps_per_pass(2, 16)
    assert s.steps_per_pass() == (2, 16)
    s.step(nsteps)
    s.sync()
    compare(case, s, shock_bubble_centres(n), nsteps, "fp32_eq64")
    rho2, _, _, T2 = s.moments_device()
    s.close()
    one = solver_for_case(case, "fp32_eq64")
    one.set_steps_per_pass(1, 0)
    one.set_tile(8)
    one.step(nsteps)
    rho1, _, _, T1 = one.moments_device()
    d = max(float((rho2 - rho1).abs().max() / rho1.abs().max()),
            float((T2 - T1).abs().max() / T1.abs().max()))
    print("two-step vs single-step fields", d, flush=True)
    assert d < 1e-6, d
    one.close()


def population_totals(solver):
    """Sum over the grid of each population of the current state, in FP64 on
    the device, read from the padded layout (16 values)."""
    cur, _ = solver.buffers()
    buf = next(b for b in solver._bufs if b.data_ptr() == cur)
    flat = buf.view(solver.storage_dtype)
    v = torch.as_strided(flat, size=(solver.ny, 16, solver.nx),
                         stride=(solver.pitch, solver.plane, 1), storage_offset=solver.origin)
    return v.double().sum(dim=(0, 2)).cpu().numpy()


def test_two_step_conserves_mass_momentum_energy_at_full_size():
    """A property that holds at any size: on a periodic grid the scheme
    conserves total mass, momentum and energy (the collision conserves them
    per cell, the Lax-Wendroff increments telescope).  2048^2 cells (304 MB
    per FP32 state: two steps per pass by default), 1000 steps: the totals
    may move only by FP32 rounding.  Then bitwise determinism of the pass."""
    n, steps = 2048, 1000
    case = smooth_case(n, n, ("periodic",) * 4, seed=13, amp=0.05)
    print(f"case {case.name} fp32_eq64 {steps} steps conservation", flush=True)
    s = solver_for_case(case, "fp32_eq64")
    assert s.steps_per_pass()[0] == 2
    vx, vy, eta = mrt.velocity_set(2.5)
    weights = np.stack([np.ones(16), vx, vy, vx * vx + vy * vy + eta * eta])
    before = weights @ population_totals(s)
    s.step(steps)
    s.sync()
    after = weights @ population_totals(s)
    mass, energy = before[0], before[3]
    drift = {"mass": abs(after[0] - mass) / mass,
             "momentum": float(np.max(np.abs(after[1:3] - before[1:3]))) / mass,
             "energy": abs(after[3] - energy) / energy}
    print("drift", drift, flush=True)
    assert all(v < 1e-6 for v in drift.values()), drift
    s.close()
    outs = []
    for _ in range(2):
        r = solver_for_case(case, "fp32_eq64")
        r.step(50)
        cur, _ = r.buffers()
        flat = next(b for b in r._bufs if b.data_ptr() == cur).view(r.storage_dtype)
        outs.append(torch.as_strided(flat, size=(r.ny, 16, r.nx), stride=(r.pitch, r.plane, 1),
                                     storage_offset=r.origin).clone())
        r.close()
    assert torch.equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp32"])
def test_plain_launches_equal_graph_replays(precision):
    """Two steps per pass: step(2) called four times launches the two-step
    kernel directly each time (the path the autotuner times), step(8)
    replays one captured graph of four passes; both must run every pass and
    give the same populations bit for bit, and an odd count (step(3) = one
    two-step pass and one single step) matches step(2) + step(1)."""
    case = smooth_case(300, 40, ("eq", "outflow", "reflect", "reflect"), seed=17)
    a = solver_for_case(case, precision)
    b = solver_for_case(case, precision)
    for s in (a, b):
        s.set_steps_per_pass(2, 8)
    for _ in range(4):
        a.step(2)
    b.step(8)
    fa, fb = a.populations(), b.populations()
    assert np.array_equal(fa, fb)
    a.step(3)
    b.step(2)
    b.step(1)
    assert np.array_equal(a.populations(), b.populations())
    # and eight steps really ran: the oracle after 11 steps
    want, p = oracle_run(case, 11)
    err = field_errors(a.moments(), mrt.macroscopic(want, p.b))
    assert all(v < 1e-5 for v in err.values()), err
    a.close()
    b.close()
