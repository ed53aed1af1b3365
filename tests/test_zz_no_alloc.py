"""The adjoint step that allocates nothing (mrt_adjoint_step_noalloc, for
callers under HIP graph capture or in loops that may not allocate): through
the C ABI against mrt_adjoint_step, which runs the same kernels with the
context's own partial-sum buffer.  Two calls in a row on the shared static
scratch, the second on a smaller grid, each bit for bit equal to the
allocating entry point; a grid with more work items than the scratch holds
is rejected before anything runs."""
import ctypes

import numpy as np
import pytest

from paper_1004_5442_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd import lib as L  # noqa: E402
from paper_1004_5442_amd.solver import Solver  # noqa: E402


def _state(sv, seed):
    """A smooth state off equilibrium (f^n) and a random lam^{n+1}, both in
    the solver's padded layout, from the library's own initialisation and
    five forward steps."""
    rng = np.random.default_rng(seed)
    ny, nx = sv.ny, sv.nx
    y, x = np.meshgrid((np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx, indexing="ij")
    rho = torch.tensor(1 + 0.05 * np.cos(2 * np.pi * (x + 2 * y)), device="cuda")
    T = torch.tensor(1 + 0.05 * np.sin(2 * np.pi * (2 * x - y)), device="cuda")
    u = torch.tensor(0.1 * np.sin(2 * np.pi * y), device="cuda")
    zero = torch.zeros_like(rho)
    f, g = sv.empty_state(), sv.empty_state()
    sv.init_buffer(rho, u, zero, T, f)
    for _ in range(5):
        sv.step_buffers(f, g)
        f, g = g, f
    lam = sv.empty_state()
    v = lam.view(sv.storage_dtype)
    v.copy_(torch.tensor(rng.standard_normal(v.numel()), device="cuda", dtype=sv.storage_dtype))
    return f, lam


def _interior(sv, buf):
    idx = (np.arange(16)[:, None, None] * sv.plane + sv.origin
           + np.arange(sv.ny)[None, :, None] * sv.pitch + np.arange(sv.nx)[None, None, :])
    return buf.view(sv.storage_dtype)[torch.as_tensor(idx.ravel(), device="cuda")]


def _both(sv, f, lam):
    out_a, out_b = sv.empty_state(), sv.empty_state()
    ds_a = torch.zeros(16, dtype=torch.float64, device="cuda")
    ds_b = torch.zeros(16, dtype=torch.float64, device="cuda")
    P = ctypes.c_void_p
    L.check(L.raw().mrt_adjoint_step(sv.handle, P(lam.data_ptr()), P(f.data_ptr()),
                                     P(out_a.data_ptr()), P(ds_a.data_ptr())), sv.handle)
    L.check(L.raw().mrt_adjoint_step_noalloc(sv.handle, P(lam.data_ptr()), P(f.data_ptr()),
                                             P(out_b.data_ptr()), P(ds_b.data_ptr())), sv.handle)
    torch.cuda.synchronize()
    return (_interior(sv, out_a), ds_a), (_interior(sv, out_b), ds_b)


@pytest.mark.parametrize("precision", ["fp32_eq64", "fp64"])
def test_noalloc_adjoint_step_equals_allocating_one(precision):
    s = W.rates(5e3, 1e4, 0.71, 1e4)
    # a grid of 3 x 300 work items, then a smaller one: the second call
    # finds the first call's partial rows in the shared scratch
    for nx, ny, seed in ((700, 300, 1), (70, 9, 2)):
        sv = Solver(nx, ny, precision)
        sv.set_params(1.4, s, 1e-4, 1.0 / nx, 1.0 / ny)
        f, lam = _state(sv, seed)
        (la, da), (lb, db) = _both(sv, f, lam)
        print(precision, nx, ny, "ds", db.tolist(), flush=True)
        assert torch.count_nonzero(da[4:]) >= 8
        assert torch.equal(la, lb)
        assert torch.equal(da, db)
        sv.close()


def test_noalloc_rejects_grid_beyond_scratch():
    # 2048 x 16384: 8 column chunks x 1024 bands of 16 rows = 8192 adjoint
    # work items, more than the 8128 the static scratch holds; rejected
    # before any kernel runs (the small buffers passed are never touched)
    sv = Solver(2048, 16384, "fp32_eq64")
    sv.set_params(1.4, W.rates(5e3, 1e4, 0.71, 1e4), 1e-4, 1.0 / 2048, 1.0 / 16384)
    small = torch.zeros(1024, dtype=torch.float32, device="cuda")
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")
    other = torch.zeros(1024, dtype=torch.float32, device="cuda")
    P = ctypes.c_void_p
    rc = L.raw().mrt_adjoint_step_noalloc(sv.handle, P(small.data_ptr()), P(small.data_ptr()),
                                          P(other.data_ptr()), P(ds.data_ptr()))
    assert rc == L.MRT_EINVAL
    msg = L.raw().mrt_last_error(sv.handle).decode()
    assert "static scratch" in msg and "8192" in msg, msg
    sv.close()
