"""GPU parity of the two alternative readings of the discretisation
(mrt_set_scheme): collide-then-stream and the nine-point Lax-Wendroff
stencil, alone and combined, against the oracle with the same options."""
import numpy as np
import pytest

from helpers import field_errors, oracle_run, smooth_case
from oracle import mrt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd.lib import MRTError  # noqa: E402
from paper_1004_5442_amd.solver import solver_for_case  # noqa: E402

VARIANTS = [(True, False), (False, True), (True, True)]
BC_SETS = [
    ("periodic", "periodic", "periodic", "periodic"),
    ("eq", "outflow", "reflect", "reflect"),
    ("reflect", "eq", "periodic", "periodic"),
    ("outflow", "reflect", "eq", "outflow"),
    ("reflect", "reflect", "reflect", "reflect"),     # every corner from two reflections
    ("eq", "reflect", "eq", "reflect"),               # EQ and reflect corners
]


@pytest.mark.parametrize("split,cross", VARIANTS)
@pytest.mark.parametrize("bc", BC_SETS)
@pytest.mark.parametrize("shape", [(150, 37), (64, 5), (1, 7), (65, 1)])
def test_variant_fp64_populations_match_oracle(split, cross, bc, shape):
    nx, ny = shape
    case = smooth_case(nx, ny, bc, seed=nx + 3 * ny)
    print(f"case {case.name} bc={bc} split={split} cross={cross}", flush=True)
    want, p = oracle_run(case, 12, split=split, lw_cross=cross)
    s = solver_for_case(case, "fp64")
    s.set_scheme(split=split, lw_cross=cross)
    s.step(12)
    got = s.populations()
    s.close()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()


@pytest.mark.parametrize("precision", ["fp32", "fp32_eq64"])
@pytest.mark.parametrize("split,cross", VARIANTS)
def test_variant_fp32_forms_match_oracle_fields(precision, split, cross):
    case = smooth_case(150, 37, ("eq", "outflow", "reflect", "reflect"), seed=3)
    print(f"case {case.name} {precision} split={split} cross={cross}", flush=True)
    want, p = oracle_run(case, 100, split=split, lw_cross=cross)
    s = solver_for_case(case, precision)
    s.set_scheme(split=split, lw_cross=cross)
    s.step(100)
    err = field_errors(s.moments(), mrt.macroscopic(want, p.b))
    s.close()
    print(err)
    assert max(err.values()) < 1e-5, err


def test_switching_back_to_the_default_scheme():
    case = smooth_case(80, 20, ("eq", "outflow", "reflect", "reflect"), seed=9)
    want, _ = oracle_run(case, 6)
    s = solver_for_case(case, "fp64")
    s.set_scheme(split=True, lw_cross=True)
    s.set_scheme()
    s.step(6)
    got = s.populations()
    s.close()
    assert np.max(np.abs(got - want)) <= 1e-12 * np.abs(want).max()


def test_explicit_buffer_calls_reject_variants():
    case = smooth_case(64, 8, ("periodic",) * 4, seed=1)
    s = solver_for_case(case, "fp64")
    s.set_scheme(split=True)
    a, b = s.empty_state(), s.empty_state()
    with pytest.raises(MRTError):
        s.step_buffers(a, b)
    s.close()
