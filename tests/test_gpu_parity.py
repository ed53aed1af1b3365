"""GPU parity: the HIP path against the FP64 oracle on the same seeded inputs.

All calls go through the C ABI (ctypes binding).  FP64 must agree to 1e-12
(relative to the field or population scale); the FP32 forms to 1e-5 on
rho, u, T (the tolerance stated for the method's FP32 form).
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
    ("eq", "outflow", "reflect", "reflect"),
    ("reflect", "eq", "periodic", "periodic"),
    ("outflow", "reflect", "eq", "outflow"),
    ("reflect", "reflect", "reflect", "reflect"),
]


@pytest.mark.parametrize("bc", BC_SETS)
@pytest.mark.parametrize("shape,rows", [((150, 37), 8), ((64, 5), 2), ((1, 7), 3), ((65, 1), 1),
                                        ((256, 12), 6), ((257, 9), 5), ((512, 3), 6)])
def test_fp64_populations_match_oracle(bc, shape, rows):
    nx, ny = shape
    case = smooth_case(nx, ny, bc, seed=nx + ny)
    print(f"case {case.name} bc={bc} rows={rows}", flush=True)
    want, p = oracle_run(case, 12)
    s = solver_for_case(case, "fp64")
    s.set_tile(rows)
    s.step(12)
    got = s.populations()
    scale = np.abs(want).max()
    assert np.max(np.abs(got - want)) <= 1e-12 * scale


@pytest.mark.parametrize("precision", ["fp32", "fp32_eq64"])
@pytest.mark.parametrize("bc", BC_SETS[:2])
def test_fp32_forms_match_oracle_fields(precision, bc):
    case = smooth_case(150, 37, bc, seed=3)
    print(f"case {case.name} {precision} bc={bc}", flush=True)
    want, p = oracle_run(case, 100)
    s = solver_for_case(case, precision)
    s.set_tile(8)
    s.step(100)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    print(precision, err)
    assert max(err.values()) < 1e-5, err


def test_sod_tube_fp64_1000_steps():
    """Plain method, FP64: the 400x4 Sod tube for 1000 steps."""
    case = W.sod_tube()
    want, p = oracle_run(case, case.nsteps)
    s = solver_for_case(case, "fp64")
    s.step(case.nsteps)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    print("sod fp64", err)
    assert max(err.values()) < 1e-12, err


@pytest.mark.parametrize("precision", ["fp32", "fp32_eq64"])
def test_riemann2d_band_fp32_vs_fp64_oracle(precision):
    """2D Riemann problem (1024 wide band of 48 rows, seed 0), 300 steps."""
    case = W.riemann2d(n=1024, ny=48, seed=0)
    want, p = oracle_run(case, 300)
    s = solver_for_case(case, precision)
    s.step(300)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    print("riemann2d", precision, err)
    assert max(err.values()) < 1e-5, err


def test_nan_sets_health_flag():
    from paper_1004_5442_amd.lib import UnstableError
    case = smooth_case(70, 9, BC_SETS[0])
    s = solver_for_case(case, "fp32_eq64")
    f = s.populations()
    f[:, 4, 33] = np.nan
    s.set_populations(f)
    s.step(1)
    with pytest.raises(UnstableError):
        s.moments()
    # the flag is cleared by the report
    s2 = solver_for_case(case, "fp32_eq64")
    s2.step(3)
    s2.moments()


def test_bitwise_deterministic():
    case = W.riemann2d(n=256, ny=64, seed=1)
    outs = []
    for _ in range(2):
        s = solver_for_case(case, "fp32_eq64")
        s.step(50)
        outs.append(s.populations())
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("precision", ["fp64", "fp32_eq64"])
def test_graph_replays_equal_plain_launches(precision):
    """mrt_step(n) for n > 1 replays captured graphs (64-step chunks plus a
    remainder graph, two start buffers); a twin grid stepped one launch at a
    time must agree bitwise after every call, with other work in between."""
    case = smooth_case(300, 40, ("reflect", "eq", "periodic", "periodic"), seed=11)
    print(f"case {case.name} {precision} graph replays", flush=True)
    a = solver_for_case(case, precision)    # plain launches
    b = solver_for_case(case, precision)    # graphs
    before = b.populations()
    b.prepare(69)                           # captures only: the state is unchanged
    assert np.array_equal(b.populations(), before)
    for n in (69, 12, 69, 3, 64):
        for _ in range(n):
            a.step(1)
        b.step(n)
        pa, pb = a.populations(), b.populations()   # synchronising host work in between
        assert np.array_equal(pa, pb), n
    a.close()
    b.close()


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp32"])
def test_fp32_forms_after_1000_steps(precision):
    """The FP32 forms against the FP64 oracle after 1000 steps (the stated
    1e-5 on rho, u, T, or twice the error of FP32 storage alone where that is
    larger), on a 1024 x 48 band of the 2D Riemann problem, with one and
    with two steps per kernel pass."""
    from helpers import fp32_tolerances
    case = W.riemann2d(n=1024, ny=48, seed=0)
    want, p = oracle_run(case, 1000)
    tol = fp32_tolerances(case, 1000, want)
    for per_pass in (1, 2):
        print(f"case {case.name} {precision} 1000 steps, {per_pass} per pass", flush=True)
        s = solver_for_case(case, precision)
        s.set_steps_per_pass(per_pass, 16)
        s.step(1000)
        err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
        s.close()
        print(precision, per_pass, "errors", err, "tolerances", tol, flush=True)
        assert all(err[k] < tol[k] for k in err), (per_pass, err, tol)
        # the stated target itself, separately from the regression bound
        assert all(v < 1e-5 for v in err.values()), (per_pass, err)
