"""GPU adjoint: per-step parity with the oracle's complex-step adjoint,
full-gradient parity with the oracle reference gradient, and the 256^2 /
500-step configuration against central finite differences."""
import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import mrt
from paper_1004_5442_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs the GPU", allow_module_level=True)

from paper_1004_5442_amd.adjoint import density_after  # noqa: E402
from paper_1004_5442_amd.solver import Solver  # noqa: E402


def _small_case(n=24, m=16, seed=0):
    rng = np.random.default_rng(seed)
    y, x = np.meshgrid((np.arange(m) + 0.5) / m, (np.arange(n) + 0.5) / n, indexing="ij")
    rho = 1 + 0.05 * np.cos(2 * np.pi * (x + 2 * y)) + 0.02 * rng.standard_normal((m, n))
    T = 1 + 0.05 * np.sin(2 * np.pi * (2 * x - y)) + 0.02 * rng.standard_normal((m, n))
    s = W.rates(5e3, 1e4, 0.71, 1e4)
    return rho, T, s, 1e-4, 1.0 / n, 1.0 / m


def _padded(solver, arr16):
    """(16, ny, nx) float64 -> device buffer in the solver's padded layout."""
    buf = solver.empty_state()
    dt = solver.storage_dtype
    v = buf.view(dt)
    idx = (np.arange(16)[:, None, None] * solver.plane + solver.origin
           + np.arange(solver.ny)[None, :, None] * solver.pitch + np.arange(solver.nx)[None, None, :])
    v[torch.as_tensor(idx.ravel(), device="cuda")] = torch.as_tensor(arr16.ravel(), device="cuda", dtype=dt)
    return buf


def _unpadded(solver, buf):
    idx = (np.arange(16)[:, None, None] * solver.plane + solver.origin
           + np.arange(solver.ny)[None, :, None] * solver.pitch + np.arange(solver.nx)[None, None, :])
    return buf.view(solver.storage_dtype)[torch.as_tensor(idx.ravel(), device="cuda")].double().cpu().numpy().reshape(16, solver.ny, solver.nx)


def test_adjoint_step_matches_oracle_fp64():
    rho, T, s, dt, dx, dy = _small_case(70, 9)
    ny, nx = rho.shape
    p = mrt.Params(gamma=1.4, s=s, dt=dt, dx=dx, dy=dy)
    rng = np.random.default_rng(1)
    f = mrt.init_populations(rho, 0 * rho, 0 * rho, T, p) * (1 + 0.01 * rng.standard_normal((16, ny, nx)))
    lam = rng.standard_normal((16, ny, nx))
    want_lam, want_ds = oadj.adjoint_step(lam, f, p)
    sv = Solver(nx, ny, "fp64")
    sv.set_params(1.4, s, dt, dx, dy)
    lam_d, f_d, out_d = _padded(sv, lam), _padded(sv, f), sv.empty_state()
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")
    sv.adjoint_step(lam_d, f_d, out_d, ds)
    got = _unpadded(sv, out_d)
    assert np.max(np.abs(got - want_lam)) <= 1e-12 * np.abs(want_lam).max()
    np.testing.assert_allclose(ds.cpu().numpy(), want_ds, rtol=1e-10, atol=1e-12 * np.abs(want_ds).max())


def test_gradient_matches_oracle_reference_fp64():
    rho, T, s, dt, dx, dy = _small_case()
    ny, nx = rho.shape
    N = 30
    p = mrt.Params(gamma=1.4, s=s, dt=dt, dx=dx, dy=dy)
    target = mrt.run(mrt.init_populations(rho, 0 * rho, 0 * rho, T + 0.01, p), p, N).sum(axis=0)
    L_ref, g_ref = oadj.density_misfit_gradient(rho, 0 * rho, 0 * rho, T, target, p, N)
    sv = Solver(nx, ny, "fp64")
    r0 = torch.tensor(rho, device="cuda", requires_grad=True)
    t0 = torch.tensor(T, device="cuda", requires_grad=True)
    st = torch.tensor(s, device="cuda", requires_grad=True)
    rhoN = density_after(r0, t0, st, sv, 1.4, dt, dx, dy, N, segment=7)
    L = 0.5 * ((rhoN - torch.tensor(target, device="cuda")) ** 2).sum()
    L.backward()
    assert L.item() == pytest.approx(L_ref, rel=1e-10)
    for name, g in (("rho", r0.grad), ("T", t0.grad), ("s", st.grad)):
        want = g_ref[name]
        got = g.detach().cpu().numpy()
        assert np.max(np.abs(got - want)) <= 1e-9 * np.abs(want).max(), name


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32_eq64", 1e-4)])
def test_adjoint_configuration_against_finite_differences(precision, tol):
    """256^2 periodic grid, 500 steps, loss = 1/2 |rho^N - rho_target|^2;
    gradient w.r.t. rho0, T0 and s from the adjoint (sqrt(N) checkpoints)
    against central differences of the FP64 forward on 32 seeded directions."""
    case, T_target = W.adjoint_problem(n=256, seed=0, nsteps=500)
    n, N = case.nx, case.nsteps
    args = (1.4, case.dt, case.dx, case.dy, N)
    s64 = Solver(n, n, "fp64")
    rho0 = torch.tensor(case.rho, device="cuda")
    T0 = torch.tensor(case.T, device="cuda")
    s0 = torch.tensor(case.s, device="cuda")
    with torch.no_grad():
        target = density_after(rho0, torch.tensor(T_target, device="cuda"), s0, s64, *args)

    def loss(r, t, s):
        with torch.no_grad():
            return float(0.5 * ((density_after(r, t, s, s64, *args) - target) ** 2).sum())

    sv = s64 if precision == "fp64" else Solver(n, n, precision)
    r = rho0.clone().requires_grad_(True)
    t = T0.clone().requires_grad_(True)
    sg = s0.clone().requires_grad_(True)
    L = 0.5 * ((density_after(r, t, sg, sv, *args) - target) ** 2).sum()
    L.backward()
    rng = np.random.default_rng(2024)
    worst = 0.0
    for d in range(32):
        dr = torch.tensor(rng.standard_normal((n, n)), device="cuda")
        dT = torch.tensor(rng.standard_normal((n, n)), device="cuda")
        # rates at s dt = 1 may move by at most ~3e-7 relative (within the
        # library's 1e-6 slack on the [0, 1/dt] interval)
        dsv = torch.tensor(rng.standard_normal(16), device="cuda") * s0 * 0.1
        ad = float((r.grad * dr).sum() + (t.grad * dT).sum() + (sg.grad * dsv).sum())
        eps = 1e-6
        fd = (loss(rho0 + eps * dr, T0 + eps * dT, s0 + eps * dsv)
              - loss(rho0 - eps * dr, T0 - eps * dT, s0 - eps * dsv)) / (2 * eps)
        rel = abs(ad - fd) / abs(fd)
        worst = max(worst, rel)
    print(precision, "worst relative FD mismatch", worst)
    assert worst < tol


def test_checkpoint_segment_does_not_change_gradient():
    rho, T, s, dt, dx, dy = _small_case(40, 24, seed=5)
    sv = Solver(40, 24, "fp32_eq64")
    grads = []
    for seg in (1, 6, 50):
        r0 = torch.tensor(rho, device="cuda", requires_grad=True)
        rhoN = density_after(r0, torch.tensor(T, device="cuda"), torch.tensor(s, device="cuda"),
                             sv, 1.4, dt, dx, dy, 37, segment=seg)
        (rhoN ** 2).sum().backward()
        grads.append(r0.grad.cpu().numpy())
    assert np.array_equal(grads[0], grads[1]) and np.array_equal(grads[1], grads[2])


@pytest.mark.parametrize("sets", [1, 2])
@pytest.mark.parametrize("nsteps,segment", [(13, 4), (12, 4), (5, 9), (1, 1), (7, 1), (8, 2)])
def test_native_checkpoint_loops_equal_explicit_steps(nsteps, segment, sets):
    """mrt_step_checkpointed / mrt_adjoint_sweep against the same work done
    one mrt_step_buffers / mrt_adjoint_step call at a time (states and lam
    bitwise, ds to rounding order), for odd and even step counts and a
    segment longer than the run; with one set of work buffers, and with two
    (the next segment recomputed on the second stream)."""
    rho, T, s, dt, dx, dy = _small_case(70, 9, seed=2)
    ny, nx = rho.shape
    sv = Solver(nx, ny, "fp32_eq64")
    sv.set_params(1.4, s, dt, dx, dy)
    r0, T0 = torch.tensor(rho, device="cuda"), torch.tensor(T, device="cuda")
    zero = torch.zeros_like(r0)
    # explicit forward: keep every state
    states = [sv.empty_state()]
    sv.init_buffer(r0, zero, zero, T0, states[0])
    for _ in range(nsteps):
        states.append(sv.empty_state())
        sv.step_buffers(states[-2], states[-1])
    # native forward with checkpoints
    f, tmp = sv.empty_state(), sv.empty_state()
    sv.init_buffer(r0, zero, zero, T0, f)
    ck = [sv.empty_state() for _ in range((nsteps + segment - 1) // segment)]
    sv.step_checkpointed(f, tmp, segment, nsteps, ck)
    torch.cuda.synchronize()
    assert torch.equal(_unpadded_t(sv, f), _unpadded_t(sv, states[nsteps]))
    for k, c in enumerate(ck):
        assert torch.equal(_unpadded_t(sv, c), _unpadded_t(sv, states[k * segment]))
    # explicit backward
    rng = np.random.default_rng(3)
    lamN = rng.standard_normal((16, ny, nx))
    lam, lam2 = _padded(sv, lamN), sv.empty_state()
    ds_ref = torch.zeros(16, dtype=torch.float64, device="cuda")
    for n in range(nsteps - 1, -1, -1):
        sv.adjoint_step(lam, states[n], lam2, ds_ref)
        lam, lam2 = lam2, lam
    # native sweep
    lamS, lamT = _padded(sv, lamN), sv.empty_state()
    work = [sv.empty_state() for _ in range(sets * (min(segment, nsteps) - 1))]
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")
    sv.adjoint_sweep(ck, segment, nsteps, work, lamS, lamT, ds)
    torch.cuda.synchronize()
    assert torch.equal(_unpadded_t(sv, lamS), _unpadded_t(sv, lam))
    # the sweep sums every step's per-wave partials before one reduction:
    # the same terms in another order
    assert torch.allclose(ds, ds_ref, rtol=1e-12, atol=1e-14 * float(ds_ref.abs().max()))
    sv.close()


def test_two_stream_sweep_equals_one_stream_sweep():
    """The sweep with two sets of work buffers (recomputation on the
    context's second stream, ordered by events) gives lam and ds bitwise
    equal to the one-set sweep, on a 300 x 40 grid over 47 steps in segments
    of 5 (ten segments, the last ragged), three calls in a row (the events
    are reused); fewer work buffers than a segment needs are refused."""
    rho, T, s, dt, dx, dy = _small_case(300, 40, seed=5)
    ny, nx = rho.shape
    sv = Solver(nx, ny, "fp32_eq64")
    sv.set_params(1.4, s, dt, dx, dy)
    r0, T0 = torch.tensor(rho, device="cuda"), torch.tensor(T, device="cuda")
    zero = torch.zeros_like(r0)
    nsteps, segment = 47, 5
    f, tmp = sv.empty_state(), sv.empty_state()
    sv.init_buffer(r0, zero, zero, T0, f)
    ck = [sv.empty_state() for _ in range((nsteps + segment - 1) // segment)]
    sv.step_checkpointed(f, tmp, segment, nsteps, ck)
    lamN = np.random.default_rng(7).standard_normal((16, ny, nx))
    out = {}
    for sets in (1, 2):
        work = [sv.empty_state() for _ in range(sets * (segment - 1))]
        for call in range(3):
            print(f"sets {sets} call {call}", flush=True)
            lam, lam2 = _padded(sv, lamN), sv.empty_state()
            ds = torch.zeros(16, dtype=torch.float64, device="cuda")
            sv.adjoint_sweep(ck, segment, nsteps, work, lam, lam2, ds)
            torch.cuda.synchronize()
            got = (_unpadded_t(sv, lam).clone(), ds.clone())
            if sets in out:
                assert torch.equal(got[0], out[sets][0]) and torch.equal(got[1], out[sets][1])
            out[sets] = got
    assert torch.equal(out[1][0], out[2][0])
    assert torch.equal(out[1][1], out[2][1])
    lam, lam2 = _padded(sv, lamN), sv.empty_state()
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(RuntimeError, match="work buffers"):
        sv.adjoint_sweep(ck, segment, nsteps, [sv.empty_state() for _ in range(segment - 2)],
                         lam, lam2, ds)
    sv.close()


def _unpadded_t(solver, buf):
    idx = (np.arange(16)[:, None, None] * solver.plane + solver.origin
           + np.arange(solver.ny)[None, :, None] * solver.pitch + np.arange(solver.nx)[None, None, :])
    return buf.view(solver.storage_dtype)[torch.as_tensor(idx.ravel(), device="cuda")]


@pytest.mark.parametrize("n", [24, 512])
def test_rate_gradient_reduction_repeats_bit_for_bit(n):
    """The rate gradient of an adjoint step is reduced in a fixed order: ten
    launches on the same input give the same ds bit for bit, on a grid of 24
    adjoint blocks and on one of 1,024, and a launch accumulates onto what
    ds holds."""
    rho, T, s, dt, dx, dy = _small_case(n, n, seed=4)
    sv = Solver(n, n, "fp32_eq64")
    sv.set_params(1.4, s, dt, dx, dy)
    r0, T0 = torch.tensor(rho, device="cuda"), torch.tensor(T, device="cuda")
    zero = torch.zeros_like(r0)
    # five steps off the initial equilibrium (at equilibrium the non-conserved
    # moments equal theirs and the rate gradient vanishes)
    f, g = sv.empty_state(), sv.empty_state()
    sv.init_buffer(r0, zero, zero, T0, f)
    for _ in range(5):
        sv.step_buffers(f, g)
        f, g = g, f
    lam = _padded(sv, np.random.default_rng(5).standard_normal((16, n, n)))
    out = sv.empty_state()
    first = None
    for rep in range(10):
        ds = torch.zeros(16, dtype=torch.float64, device="cuda")
        sv.adjoint_step(lam, f, out, ds)
        torch.cuda.synchronize()
        if first is None:
            first = ds.clone()
            print("ds", first.tolist(), flush=True)
            assert torch.count_nonzero(first[4:]) >= 8 and torch.count_nonzero(first[:4]) == 0
        assert torch.equal(ds, first), (rep, ds, first)
    ds = first.clone()
    sv.adjoint_step(lam, f, out, ds)
    torch.cuda.synchronize()
    assert torch.allclose(ds, 2 * first, rtol=1e-14, atol=0), (ds, first)
    sv.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("fp32_eq64", 1e-6)])
def test_init_adjoint_all_four_gradients_match_oracle(precision, tol):
    """mrt_init_adjoint's g_rho, g_ux, g_uy and g_T against the oracle's
    init_adjoint (complex step of init_populations) on a moving state whose
    two velocity components differ, so that a swapped or mis-indexed
    velocity gradient fails.  FP64 at 1e-12 of each gradient's scale; FP32
    storage only rounds lam0 on the way in (the Jacobian is FP64 there)."""
    rng = np.random.default_rng(21)
    ny, nx = 11, 67
    rho = 1 + 0.1 * rng.standard_normal((ny, nx))
    T = 1 + 0.1 * rng.standard_normal((ny, nx))
    ux = 0.3 + 0.2 * rng.standard_normal((ny, nx))
    uy = -0.2 + 0.2 * rng.standard_normal((ny, nx))
    s = W.rates(5e3, 1e4, 0.71, 1e4)
    p = mrt.Params(gamma=1.4, s=s, dt=1e-4, dx=1.0 / nx, dy=1.0 / ny)
    lam0 = rng.standard_normal((16, ny, nx))
    sv = Solver(nx, ny, precision)
    sv.set_params(1.4, s, 1e-4, 1.0 / nx, 1.0 / ny)
    lam_d = _padded(sv, lam0)
    # the oracle sees lam0 as the device stores it
    lam_used = _unpadded(sv, lam_d)
    want = oadj.init_adjoint(lam_used, rho, ux, uy, T, p)
    dev = [torch.tensor(a, device="cuda") for a in (rho, ux, uy, T)]
    outs = [torch.full((ny, nx), np.nan, dtype=torch.float64, device="cuda") for _ in range(4)]
    sv.init_adjoint(lam_d, *dev, g_rho=outs[0], g_ux=outs[1], g_uy=outs[2], g_T=outs[3])
    torch.cuda.synchronize()
    for k, name in enumerate(("rho", "ux", "uy", "T")):
        got = outs[k].cpu().numpy()
        err = np.max(np.abs(got - want[k])) / np.max(np.abs(want[k]))
        print(precision, name, "relative error", err, flush=True)
        assert err <= tol, (name, err)
    sv.close()


def test_backward_uses_the_parameters_of_its_own_forward():
    """Two forwards with different rates on one solver, then backward of the
    first: the gradient is that of the first forward's parameters (the
    adjoint sweep re-applies them), equal bit for bit to a run without the
    second forward."""
    rho, T, s, dt, dx, dy = _small_case(32, 16, seed=9)
    sv = Solver(32, 16, "fp64")
    s2 = np.array(s) * 0.5

    def grad(with_second):
        r0 = torch.tensor(rho, device="cuda", requires_grad=True)
        rhoN = density_after(r0, torch.tensor(T, device="cuda"), torch.tensor(s, device="cuda"),
                             sv, 1.4, dt, dx, dy, 12, segment=4)
        if with_second:
            with torch.no_grad():
                density_after(r0.detach(), torch.tensor(T, device="cuda"),
                              torch.tensor(s2, device="cuda"), sv, 1.4, dt, dx, dy, 12, segment=4)
        (rhoN ** 2).sum().backward()
        torch.cuda.synchronize()
        return r0.grad.cpu().numpy()

    a = grad(False)
    b = grad(True)
    assert np.array_equal(a, b)
    # parameters are set again only where they changed: a backward right
    # after its own forward sets none (setting them waits for the stream)
    calls = []
    orig = Solver.set_params

    def counted(self, *args, **kw):
        calls.append(args)
        return orig(self, *args, **kw)

    Solver.set_params = counted
    try:
        c = grad(False)      # the last backward left s set: none
        assert len(calls) == 0, calls
        d = grad(False)
        assert len(calls) == 0, calls
        e = grad(True)       # the second forward (s2), then the backward (s): two
        assert len(calls) == 2, calls
    finally:
        Solver.set_params = orig
    assert np.array_equal(a, c) and np.array_equal(a, d) and np.array_equal(a, e)
    sv.close()
