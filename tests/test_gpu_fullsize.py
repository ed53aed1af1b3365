"""GPU parity at full size, in the launch configuration the benchmark times.

The 4096^2 shock-bubble grid (FP32 storage: 1.15 GB per population buffer,
so the kernels take their non-temporal store path; both precisions run two
steps per pass by default there, and the one-step kernel is checked too) and
the 1024^2 2D Riemann grid (cache-resident, cached stores) run a few steps on
the GPU; the
oracle evaluates small windows around sampled cells (the shock front, the
bubble edge, every kind of boundary, the corners) one by one
(``mrt.evolve_window``: a window of the initial fields grown by one cell per
step, so every sampled cell's dependence cone is inside it); both grids
again after 100 steps against 206 x 206 windows.  A longer run
checks a property that holds at any size: the shock-bubble problem is
mirror-symmetric about y = 1/2, so the GPU fields must be too, to rounding.
"""
import numpy as np
import pytest

from helpers import field_errors, fp32_tolerances, oracle_params, oracle_run
from oracle import mrt
from paper_1004_5442_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd.solver import solver_for_case  # noqa: E402

HEADLINE_BAND_ROWS_2 = 32    # the benchmark's 4096^2 FP32 run: two steps per pass, 32-row bands
FP64_BAND_ROWS_2 = 64        # its FP64 run (the library's default for FP64 at this size)
HEADLINE_TILE_ROWS = 8       # its one-step-per-pass runs (FP64, and FP32 for comparison)
NSTEPS = 6                   # steps before sampling (window margin = NSTEPS)
PATCH = 6                    # sampled patch: PATCH x PATCH cells


def device_samples(solver, xs, ys):
    """Populations of the current buffer at cells (xs[k], ys[k]), float64
    (16, len(xs)); gathers on the device and copies only the samples."""
    cur, _ = solver.buffers()
    buf = next(b for b in solver._bufs if b.data_ptr() == cur)
    flat = buf.view(solver.storage_dtype)
    xs = torch.as_tensor(np.asarray(xs), dtype=torch.int64, device="cuda")
    ys = torch.as_tensor(np.asarray(ys), dtype=torch.int64, device="cuda")
    i = torch.arange(16, dtype=torch.int64, device="cuda")[:, None]
    idx = i * solver.plane + solver.origin + ys[None, :] * solver.pitch + xs[None, :]
    return flat[idx].double().cpu().numpy()


def patches(case, centres):
    """(x0, x1, y0, y1) patches of PATCH x PATCH cells around the centres,
    clipped to the grid."""
    out = []
    for cx, cy in centres:
        x0 = int(np.clip(cx - PATCH // 2, 0, case.nx - PATCH))
        y0 = int(np.clip(cy - PATCH // 2, 0, case.ny - PATCH))
        out.append((x0, x0 + PATCH, y0, y0 + PATCH))
    return out


def oracle_patch(case, p, patch, nsteps):
    x0, x1, y0, y1 = patch
    f, (wx0, wx1, wy0, wy1) = mrt.evolve_window(case.rho, case.ux, case.uy, case.T, p,
                                                x0 - nsteps, x1 + nsteps, y0 - nsteps,
                                                y1 + nsteps, nsteps)
    sub = f[:, y0 - wy0:y1 - wy0, x0 - wx0:x1 - wx0]
    assert np.isfinite(sub).all()
    return sub


def compare(case, solver, centres, nsteps, precision):
    p = oracle_params(case)
    got_all, want_all = [], []
    for patch in patches(case, centres):
        x0, x1, y0, y1 = patch
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        got = device_samples(solver, xx.ravel(), yy.ravel()).reshape(16, PATCH, PATCH)
        got_all.append(got)
        want_all.append(oracle_patch(case, p, patch, nsteps))
    got = np.concatenate(got_all, axis=2)
    want = np.concatenate(want_all, axis=2)
    if precision == "fp64":
        err = np.max(np.abs(got - want)) / np.abs(want).max()
        print(case.name, precision, "population error", err, flush=True)
        assert err <= 1e-12
    else:
        err = field_errors(mrt.macroscopic(got, p.b), mrt.macroscopic(want, p.b))
        print(case.name, precision, err, flush=True)
        assert max(err.values()) < 1e-5, err


def shock_bubble_centres(n):
    sx = int(0.1 * n)                  # shock front
    bx, by, br = int(0.25 * n), n // 2, int(0.1 * n)
    # bubble-edge points on the column seams of the 256-column work items
    seam = 3 * n // 16
    seam_y = by + int(np.sqrt(br * br - (bx - seam) ** 2))
    return [(sx, n // 2), (sx, 1), (sx, n - 2),          # shock, where it meets the walls
            (bx - br, by), (bx + br, by),                # bubble edge
            (bx, by + br), (bx, by - br), (seam, seam_y),  # bubble edge on item seams
            (0, n // 3), (n - 1, 2 * n // 3),            # inflow, outflow sides
            (n // 2, 0), (n // 2, n - 1),                # reflecting walls
            (0, 0), (n - 1, n - 1), (0, n - 1), (n - 1, 0)]   # corners


@pytest.mark.parametrize("precision,per_pass,rows", [("fp32_eq64", 2, HEADLINE_BAND_ROWS_2),
                                                     ("fp32_eq64", 1, HEADLINE_TILE_ROWS),
                                                     ("fp64", 2, FP64_BAND_ROWS_2),
                                                     ("fp64", 1, HEADLINE_TILE_ROWS)])
def test_shock_bubble_4096_sampled(precision, per_pass, rows):
    n = 4096
    case = W.shock_bubble(n=n)
    print(f"case {case.name} {precision} {per_pass} steps per pass, {rows}-row bands", flush=True)
    s = solver_for_case(case, precision)
    if per_pass == 2:
        if precision == "fp64":
            assert s.steps_per_pass() == (2, FP64_BAND_ROWS_2)    # the default here
        s.set_steps_per_pass(2, rows)
    else:
        s.set_steps_per_pass(1, 0)
        s.set_tile(rows)
    s.step(NSTEPS)
    s.sync()
    compare(case, s, shock_bubble_centres(n), NSTEPS, precision)
    s.close()


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp64"])
def test_riemann2d_1024_sampled_autotuned(precision):
    n = 1024
    case = W.riemann2d(n=n, seed=0)
    print(f"case {case.name} {precision} autotuned", flush=True)
    s = solver_for_case(case, precision)
    s.autotune(4)        # restores the initial state
    s.step(NSTEPS)
    s.sync()
    c = n // 2
    centres = [(c, c), (c - 1, c + 1), (c, 0), (c, n - 1), (0, c), (n - 1, c),
               (0, 0), (n - 1, n - 1), (255, 700), (768, 300)]
    compare(case, s, centres, NSTEPS, precision)
    s.close()


_WINDOWS = {}


def _oracle_windows(case, centres, nsteps):
    """The oracle's patches after nsteps steps, each evolved on its own
    window grown by nsteps cells (cached per case name and step count)."""
    key = (case.name, nsteps, tuple(centres))
    if key not in _WINDOWS:
        p = oracle_params(case)
        _WINDOWS[key] = [oracle_patch(case, p, patch, nsteps) for patch in patches(case, centres)]
    return _WINDOWS[key]


def compare_long(case, solver, centres, nsteps, precision):
    """As compare, after a longer run: FP64 populations at 1e-12 of their
    scale, the FP32 forms' fields at the stated 1e-5."""
    p = oracle_params(case)
    want = np.concatenate(_oracle_windows(case, centres, nsteps), axis=2)
    got_all = []
    for x0, x1, y0, y1 in patches(case, centres):
        yy, xx = np.meshgrid(np.arange(y0, y1), np.arange(x0, x1), indexing="ij")
        got_all.append(device_samples(solver, xx.ravel(), yy.ravel()).reshape(16, PATCH, PATCH))
    got = np.concatenate(got_all, axis=2)
    if precision == "fp64":
        err = np.max(np.abs(got - want)) / np.abs(want).max()
        print(case.name, precision, nsteps, "steps: population error", err, flush=True)
        assert err <= 1e-12
    else:
        err = field_errors(mrt.macroscopic(got, p.b), mrt.macroscopic(want, p.b))
        print(case.name, precision, nsteps, "steps:", err, flush=True)
        assert max(err.values()) < 1e-5, err


@pytest.mark.parametrize("precision", ["fp64", "fp32_eq64", "fp32"])
def test_riemann2d_1024_sampled_after_100_steps(precision):
    """The 2D Riemann workload at its configured size in its autotuned
    launch, after 100 steps, on patches where all four states meet, on a
    quadrant interface, and where interfaces meet two outflow sides, against
    the oracle's windowed evaluation (windows of up to 206 x 206 cells)."""
    n, nsteps = 1024, 100
    case = W.riemann2d(n=n, seed=0)
    print(f"case {case.name} {precision} autotuned, {nsteps} steps", flush=True)
    s = solver_for_case(case, precision)
    s.autotune(4)
    s.step(nsteps)
    s.sync()
    c = n // 2
    compare_long(case, s, [(c, c), (c, 300), (0, c), (c, n - 1)], nsteps, precision)
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_eq64"])
def test_shock_bubble_4096_sampled_after_100_steps(precision):
    """The shock-bubble workload at 4096^2 in the launch the benchmark times
    for each precision (two steps per pass, 32-row bands in FP32 storage,
    64-row in FP64), after 100 steps,
    on patches at the shock front, where it meets a wall, on the bubble edge
    and at the inflow and outflow sides, against the oracle's windowed
    evaluation (windows of up to 206 x 206 cells)."""
    n, nsteps = 4096, 100
    case = W.shock_bubble(n=n)
    print(f"case {case.name} {precision} two steps per pass, {nsteps} steps", flush=True)
    rows = FP64_BAND_ROWS_2 if precision == "fp64" else HEADLINE_BAND_ROWS_2
    s = solver_for_case(case, precision)
    s.set_steps_per_pass(2, rows)
    assert s.steps_per_pass() == (2, rows)
    s.step(nsteps)
    s.sync()
    bx, by, br = int(0.25 * n), n // 2, int(0.1 * n)
    centres = [(int(0.1 * n) + 8, n // 2), (int(0.1 * n) + 8, 1), (bx - br, by), (bx, by + br),
               (0, n // 3), (n - 1, 2 * n // 3)]
    compare_long(case, s, centres, nsteps, precision)
    s.close()


def symmetry_tolerances(precision, steps):
    """FP64: 1e-10 (rounding only).  FP32 storage: the mirror image of a
    field differs from it by at most twice the field's error, so the
    tolerance is twice the FP32-storage error, estimated by the oracle with
    float32-rounded populations on the centre band (4 rows through the
    bubble, where the shock is one-dimensional), with a further factor 4 for
    the shock-wall junctions the band does not contain (fp32_tolerances
    already returns twice the band error)."""
    if precision == "fp64":
        return {"rho": 1e-10, "u": 1e-10, "T": 1e-10}
    band = W.shock_bubble(n=4096, ny=4)
    want, _ = oracle_run(band, steps)
    return {k: 4.0 * v for k, v in fp32_tolerances(band, steps, want).items()}


@pytest.mark.parametrize("precision", ["fp64", "fp32_eq64"])
def test_shock_bubble_4096_mirror_symmetry(precision):
    """rho, u_x, T even and u_y odd under y -> 1 - y, after 200 steps."""
    n, steps = 4096, 200
    tol = symmetry_tolerances(precision, steps)
    case = W.shock_bubble(n=n)
    print(f"case {case.name} {precision} {steps} steps symmetry, tol {tol}", flush=True)
    s = solver_for_case(case, precision)
    if precision == "fp64":
        s.set_tile(HEADLINE_TILE_ROWS)
    else:
        s.set_steps_per_pass(2, HEADLINE_BAND_ROWS_2)
    s.step(steps)
    rho, ux, uy, T = s.moments_device()
    s.sync()
    s.close()
    scale_u = float(torch.sqrt(T.max()))
    err = {"rho": float((rho - rho.flip(0)).abs().max() / rho.abs().max()),
           "T": float((T - T.flip(0)).abs().max() / T.abs().max()),
           "u": max(float((ux - ux.flip(0)).abs().max()),
                    float((uy + uy.flip(0)).abs().max())) / scale_u}
    print("symmetry", precision, err, flush=True)
    assert all(err[k] < tol[k] for k in err), (err, tol)
    # and the run moved: the shock has advanced several cells
    assert float(rho[n // 2, int(0.1 * n) + 10]) > 1.5


@pytest.mark.parametrize("per_pass", [2, 1])
def test_largest_grids_use_the_full_32_bit_offset_range(per_pass):
    """12000 x 12000 cells, FP32 storage: 2.36e9 elements per state, past
    the 2^31 that signed 32-bit row offsets would reach, with the two-step
    kernel (the default at this size) and the one-step kernel.  A few
    steps, then patches at the shock, the bubble, the walls and the corners
    against the oracle."""
    n = 12000
    case = W.shock_bubble(n=n)
    print(f"case {case.name} fp32_eq64 {NSTEPS} steps, {per_pass} per pass", flush=True)
    s = solver_for_case(case, "fp32_eq64")
    assert s.population_bytes() > 4 * 2 ** 31
    assert s.steps_per_pass()[0] == 2
    if per_pass == 1:
        s.set_steps_per_pass(1, 0)
        s.set_tile(HEADLINE_TILE_ROWS)
    s.step(NSTEPS)
    s.sync()
    centres = [(int(0.1 * n), n // 2), (int(0.1 * n), 0), (int(0.15 * n), n // 2),
               (n // 2, n - 1), (0, 0), (n - 1, n - 1), (n - 1, 0), (0, n - 1)]
    compare(case, s, centres, NSTEPS, "fp32_eq64")
    s.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_eq64"])
def test_large_grid_with_reflecting_walls_on_every_side(precision):
    """Above 2^22 cells the reflecting-wall ghosts come from the separate
    ghost pass (smaller grids write them in the step kernel): a 2048 x 2049
    2D Riemann grid (FP32: 304 MB per state, so two steps per pass; an odd
    step count, so the last step is a one-step pass) with reflecting walls
    on all four sides, sampled at the walls, the corners and the quadrant
    interfaces after a few steps."""
    import dataclasses
    base = W.riemann2d(n=2048, seed=4)
    rows = 2049
    pad = lambda a: np.concatenate([a, a[-1:]], axis=0)
    case = dataclasses.replace(base, name="riemann2d_2048x2049_reflect", ny=rows, rho=pad(base.rho),
                               ux=pad(base.ux), uy=pad(base.uy), T=pad(base.T),
                               bc=("reflect",) * 4)
    assert case.cells > 1 << 22
    print(f"case {case.name} {precision} ghost pass", flush=True)
    s = solver_for_case(case, precision)
    s.set_tile(HEADLINE_TILE_ROWS)
    if precision != "fp64":
        assert s.steps_per_pass()[0] == 2
    s.step(NSTEPS + 1)
    s.sync()
    nx, ny = case.nx, case.ny
    centres = [(0, ny // 3), (nx - 1, 2 * ny // 3), (nx // 3, 0), (2 * nx // 3, ny - 1),
               (0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, ny // 2),
               (nx // 2, 0), (0, ny // 2)]
    compare(case, s, centres, NSTEPS + 1, precision)
    s.close()


def shock_position(row, mid):
    """x (in cells, sub-cell by linear interpolation) where the density of a
    row first falls below `mid` coming from the post-shock side."""
    r = row.double().cpu().numpy()
    i = int(np.argmax(r < mid))
    assert i > 0
    return (i - 1) + (r[i - 1] - mid) / (r[i - 1] - r[i])


def test_shock_bubble_shock_moves_at_the_rankine_hugoniot_speed():
    """Physics at full size on the benchmark's path (4096^2, FP32 storage,
    two steps per pass), over the workload's 5000 steps: away from the
    bubble the Mach-5 shock is planar and moves at U_s = M sqrt(gamma T1)
    (pre-shock gas at rest).  Its position on the row y = 1/4 after 400, 2000
    and 5000 steps gives the speed (the bubble, first struck near step 2180,
    sends disturbances at most ~0.06 sideways by step 5000, short of that row
    0.15 away); the run stays healthy throughout."""
    n = 4096
    case = W.shock_bubble(n=n)
    gamma, T1 = case.gamma, 0.6
    u_s = 5.0 * np.sqrt(gamma * T1)
    rho_post = case.meta["post"][0]
    mid = 0.5 * (rho_post + 1.0)
    s = solver_for_case(case, "fp32_eq64")
    assert s.steps_per_pass()[0] == 2
    xs = []
    for steps in (400, 1600, 3000):
        print(f"case {case.name} fp32_eq64 +{steps} steps", flush=True)
        s.step(steps)
        rho = s.moments_device()[0]
        xs.append(shock_position(rho[n // 4], mid))
    s.sync()          # raises if any step went unhealthy
    s.close()
    speeds = [(xs[1] - xs[0]) / n / (1600 * case.dt), (xs[2] - xs[1]) / n / (3000 * case.dt)]
    print("shock positions (cells)", xs, "speeds", speeds, "Rankine-Hugoniot", u_s, flush=True)
    assert all(abs(v / u_s - 1.0) < 5e-3 for v in speeds), (speeds, u_s)


def test_shock_bubble_fp32_against_fp64_50_steps():
    """The workload's FP64 spot check: the whole 4096^2 field after 50 steps
    on the benchmark's path (FP32 storage, two steps per pass) against the
    FP64 kernel on the same input, per field, within the FP32 tolerance of
    this workload (twice the FP32-storage error the oracle shows on its
    centre band, at least 1e-5)."""
    n, steps = 4096, 50
    band = W.shock_bubble(n=n, ny=4)
    want, _ = oracle_run(band, steps)
    tol = fp32_tolerances(band, steps, want)
    case = W.shock_bubble(n=n)
    fields = {}
    for precision in ("fp64", "fp32_eq64"):
        print(f"case {case.name} {precision} {steps} steps", flush=True)
        s = solver_for_case(case, precision)
        s.step(steps)
        fields[precision] = [f.double() for f in s.moments_device()]
        s.sync()
        s.close()
    r64, u64, v64, T64 = fields["fp64"]
    r32, u32, v32, T32 = fields["fp32_eq64"]
    sp = max(float(torch.sqrt(u64 * u64 + v64 * v64).max()), float(torch.sqrt(T64.max())))
    err = {"rho": float((r32 - r64).abs().max() / r64.abs().max()),
           "u": max(float((u32 - u64).abs().max()), float((v32 - v64).abs().max())) / sp,
           "T": float((T32 - T64).abs().max() / T64.abs().max())}
    print("fp32 vs fp64", err, "tolerance", tol, flush=True)
    assert all(err[k] < tol[k] for k in err), (err, tol)


_RIEMANN2D = {}


def _riemann2d_2000():
    """The 2D Riemann workload as configured (1024^2, 2000 steps) in FP64,
    FP32 storage with FP64 collision and pure FP32 (autotuned launches); the
    FP32 forms' per-field errors against the FP64 kernel over the whole
    field, and the FP32-storage tolerances of a 1024 x 8 band of it."""
    if not _RIEMANN2D:
        n, steps = 1024, 2000
        band = W.riemann2d(n=n, ny=8, seed=0)
        want, _ = oracle_run(band, steps)
        _RIEMANN2D["tol"] = fp32_tolerances(band, steps, want)
        case = W.riemann2d(n=n, seed=0)
        fields = {}
        for precision in ("fp64", "fp32_eq64", "fp32"):
            print(f"case {case.name} {precision} {steps} steps", flush=True)
            s = solver_for_case(case, precision)
            s.autotune(4)
            s.step(steps)
            fields[precision] = [f.double() for f in s.moments_device()]
            s.sync()
            s.close()
        r64, u64, v64, T64 = fields["fp64"]
        sp = max(float(torch.sqrt(u64 * u64 + v64 * v64).max()), float(torch.sqrt(T64.max())))
        for precision in ("fp32_eq64", "fp32"):
            r, u, v, T = fields[precision]
            _RIEMANN2D[precision] = {
                "rho": float((r - r64).abs().max() / r64.abs().max()),
                "u": max(float((u - u64).abs().max()), float((v - v64).abs().max())) / sp,
                "T": float((T - T64).abs().max() / T64.abs().max())}
            print(precision, "vs fp64", _RIEMANN2D[precision], flush=True)
    return _RIEMANN2D


def test_riemann2d_1024_fp32_forms_against_fp64_2000_steps():
    """Regression bound of both FP32 forms on the 2D Riemann workload as
    configured: FP32 storage with FP64 collision within twice the
    FP32-storage error the oracle shows on a 1024 x 8 band of it after 2000
    steps (at least 1e-5); pure FP32, whose collision arithmetic also rounds
    to FP32 (measured 1.3 to 2.7 times the other form's error here), within
    four times it."""
    res = _riemann2d_2000()
    for precision, factor in (("fp32_eq64", 1.0), ("fp32", 2.0)):
        err = res[precision]
        bound = {k: factor * v for k, v in res["tol"].items()}
        print(precision, "vs fp64", err, "tolerance", bound, flush=True)
        assert all(err[k] < bound[k] for k in err), (precision, err, bound)


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp32"])
def test_riemann2d_1024_stated_tolerance(precision):
    """The stated target itself, per field and form: 1e-5 relative on rho, u
    and T after the configured 2000 steps of the 2D Riemann workload, against
    the FP64 kernel (whose own distance to the oracle is at the 1e-12 level
    on the sampled patches).  Measured: FP32 storage with FP64 collision
    rho 5.9e-6, u 6.2e-6, T 7.5e-6; pure FP32 rho 7.3e-6, u 6.4e-6, T 8.5e-6
    (it missed the target at 1.1e-5 / 1.7e-5 while its FP32 transforms let
    the compiler fuse products across statements, differently per row)."""
    err = _riemann2d_2000()[precision]
    print(precision, "stated-tolerance check", err, flush=True)
    assert all(v < 1e-5 for v in err.values()), (precision, err)
