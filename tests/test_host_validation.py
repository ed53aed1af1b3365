"""Argument validation of the C ABI, exercised on the CPU: every call here
is rejected before the library touches the GPU (sizes, boundary kinds,
precision, scheme parameters, NULL handles)."""
import ctypes
from ctypes import byref, c_int, c_void_p

import numpy as np
import pytest

L = pytest.importorskip("paper_1004_5442_amd.lib")
lib = L.raw()


def _init(nx, ny, prec=2, bc=(0, 0, 0, 0)):
    h = c_void_p()
    rc = lib.mrt_init_grid(byref(h), nx, ny, prec, (c_int * 4)(*bc), None, None)
    return rc, h


def test_population_bytes_follow_the_layout():
    for nx, ny, prec in ((1, 1, 0), (300, 7, 2), (4096, 4096, 1)):
        sub = (nx + 3 + 255) // 256 * 256
        elems = (ny + 2) * (16 * sub + 256) + 512
        assert lib.mrt_population_bytes(nx, ny, prec) == elems * (8 if prec == 0 else 4)
    assert lib.mrt_population_bytes(0, 5, 2) == 0
    assert lib.mrt_population_bytes(5, 0, 2) == 0
    # 2^32 elements per state is the limit of the kernels' 32-bit offsets
    assert lib.mrt_population_bytes(16000, 16000, 2) > 0
    assert lib.mrt_population_bytes(16384, 16384, 2) == 0


@pytest.mark.parametrize("nx,ny,prec,bc", [
    (0, 8, 2, (0, 0, 0, 0)),            # empty grid
    (8, 0, 2, (0, 0, 0, 0)),
    (16384, 16384, 2, (0, 0, 0, 0)),    # beyond 32-bit offsets
    (8, 8, 3, (0, 0, 0, 0)),            # unknown precision
    (8, 8, -1, (0, 0, 0, 0)),
    (8, 8, 2, (0, 1, 0, 0)),            # periodic x-lo without periodic x-hi
    (8, 8, 2, (1, 1, 2, 0)),            # periodic y-hi alone
    (8, 8, 2, (4, 1, 0, 0)),            # unknown boundary kind
])
def test_init_grid_rejects(nx, ny, prec, bc):
    rc, h = _init(nx, ny, prec, bc)
    assert rc == L.MRT_EINVAL and not h.value


def test_init_grid_needs_an_output_pointer():
    assert lib.mrt_init_grid(None, 8, 8, 2, (c_int * 4)(0, 0, 0, 0), None, None) == L.MRT_EINVAL


def _instance(nx=64, ny=4, bc=(1, 1, 0, 0), **kw):
    inst = L.Instance()
    inst.nx, inst.ny = nx, ny
    for k in range(4):
        inst.bc[k] = bc[k]
    s = np.zeros(16)
    s[4:] = 1e4
    h = 1.0 / max(nx, 1)
    args = dict(gamma=1.4, s=s, dt=1e-5, dx=h, dy=h, Pr=0.0, side_state=None, eta0=2.5)
    args.update(kw)
    inst.params = L.make_params(**args)
    return inst


def _batch(*insts, prec=2):
    arr = (L.Instance * len(insts))(*insts)
    h = c_void_p()
    rc = lib.mrt_batch_create(byref(h), len(insts), arr, prec, None)
    return rc, h


@pytest.mark.parametrize("kw", [
    dict(gamma=1.0),                                   # gamma must exceed 1 (b = 2/(gamma-1))
    dict(gamma=2.5),                                   # gamma > 2: negative extra dof
    dict(dt=0.0),
    dict(dx=-1.0),
    dict(eta0=3.0),                                    # eta is 5/2 in this model
    dict(s=np.r_[np.zeros(4), np.full(12, 2e5)]),      # s dt = 2 > 1
    dict(s=np.r_[np.zeros(4), -1.0, np.full(11, 1e4)]),  # negative rate
    dict(Pr=-1.0),
    dict(Pr=0.71, s=np.r_[np.zeros(4), 1e4, 1e4, 2e4, np.full(9, 1e4)]),  # Pr > 0 needs s_7 == s_6
    dict(side_state=[(0.0, 0.0, 0.0, 1.0)] * 4),       # EQ side state with rho = 0
    dict(side_state=[(1.0, 0.0, 0.0, -1.0)] * 4),      # EQ side state with T < 0
])
def test_parameter_validation(kw):
    rc, h = _batch(_instance(**kw))
    assert rc == L.MRT_EINVAL and not h.value


def test_batch_shape_validation():
    assert _batch(_instance(nx=0))[0] == L.MRT_EINVAL
    assert _batch(_instance(bc=(0, 1, 0, 0)))[0] == L.MRT_EINVAL
    assert _batch(_instance(), prec=5)[0] == L.MRT_EINVAL
    h = c_void_p()
    assert lib.mrt_batch_create(byref(h), 0, None, 2, None) == L.MRT_EINVAL
    # one bad instance among good ones rejects the batch
    assert _batch(_instance(), _instance(gamma=0.5), _instance())[0] == L.MRT_EINVAL


def test_null_handles_are_rejected():
    p = L.make_params(1.4, np.zeros(16), 1e-5, 1e-2, 1e-2)
    assert lib.mrt_set_params(None, byref(p)) == L.MRT_EINVAL
    assert lib.mrt_step(None, 1) == L.MRT_EINVAL
    assert lib.mrt_sync(None) == L.MRT_EINVAL
    assert lib.mrt_set_scheme(None, 1) == L.MRT_EINVAL
    assert lib.mrt_set_tile(None, 4, 0) == L.MRT_EINVAL
    assert lib.mrt_adjoint_step(None, None, None, None, None) == L.MRT_EINVAL
    assert lib.mrt_batch_step(None, 1) == L.MRT_EINVAL
    assert lib.mrt_set_steps_per_pass(None, 2, 0) == L.MRT_EINVAL
    assert lib.mrt_get_steps_per_pass(None, None, None) == L.MRT_EINVAL
    assert lib.mrt_batch_set_steps_per_pass(None, 2, 0) == L.MRT_EINVAL
    assert lib.mrt_batch_get_steps_per_pass(None, None, None) == L.MRT_EINVAL
    assert lib.mrt_prepare_steps(None, 4) == L.MRT_EINVAL
    assert lib.mrt_autotune(None, 4) == L.MRT_EINVAL
    assert lib.mrt_last_error(None) == b"NULL context"
    assert lib.mrt_batch_last_error(None) == b"NULL batch"
    lib.mrt_destroy(None)
    lib.mrt_batch_destroy(None)


def test_host_utilities_validate():
    out = np.empty(16)
    d = out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.mrt_host_transform(7, d, d) == L.MRT_EINVAL
    assert lib.mrt_host_transform(0, None, d) == L.MRT_EINVAL
    assert lib.mrt_host_equilibrium(1.0, 1.0, 0.0, 0.0, 1.0, d) == L.MRT_EINVAL
