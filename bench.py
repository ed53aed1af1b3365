"""Throughput of the D2V16 MRT FD-LB step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W]

One "step" is one time step of the whole hot path (ghosts, moments,
equilibrium, M / relax / Minv collision, Lax-Wendroff convection, forward
Euler) over the whole grid of the headline workload: the 4096 x 4096 Mach-5
shock hitting a dense bubble, FP32 populations with FP64 collision
(MRT_FP32_EQ64), run as the library runs it by default at this size: two
time steps per kernel pass (32-row bands).  value = MLUPS (million
lattice-site updates per second), populations already resident in HBM.
Extra fields report the one-step-per-pass kernel and the FP64 form on the
same grid, the 1024^2 2D Riemann problem, the batched shock tubes and the
adjoint step, the roofline of the step kernel, and the oracle's CPU rate on a
bounded sample.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0               # MI355X HBM3E, published
BYTES_PER_SITE = {"fp64": 256, "fp32": 128, "fp32_eq64": 128}   # 16 reads + 16 writes
HEADLINE_PER_PASS = 2               # time steps per kernel pass (the default at this size)
HEADLINE_BAND_ROWS = 32             # band height of the two-step kernel (the default here)
FP64_BAND_ROWS = 64                 # the same for FP64 storage (one block per CU)
HEADLINE_TILE_ROWS = 8              # the one-step kernel's band height for this grid

# HBM traffic of one step2_kernel launch (two steps) on the headline
# workload, from two rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per
# dispatch, mean over the step dispatches) of
#   bench.py --steps 10 --warmup 2 --no-cpu --no-extra --copy-calibration
# each scaled by what the same counter reads, in the same run, for a plain
# 1 GiB device copy (FETCH_SIZE 524,305.0 KiB, WRITE_SIZE 1,048,576 KiB for
# 1,048,576 KiB moved: factors 2.0 and 1.0).  Valid only for the step-kernel
# sources with this digest and this band height; otherwise the roofline
# reports traffic = null (comments are not hashed).
MEASURED_TRAFFIC = {
    "digest": "0bebd163d542c0e9538710b7c4ea9114b63e312a3daf1b6be539b68fc505a000",
    "band_rows": HEADLINE_BAND_ROWS,
    "fetch_kib": 747054.0, "fetch_copy_kib": 524304.7,
    "write_kib": 1049089.3, "write_copy_kib": 1048576.0,
}
STEP_HEADERS = ("mrt_transform.h", "mrt_transform_impl.inc", "mrt_internal.h")


def _code_only(text: str) -> str:
    """C++ source without comments, whitespace collapsed (so that editing a
    comment does not invalidate a measurement)."""
    import re
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    return " ".join(text.split())


def kernel_digest() -> str:
    """sha256 over what decides the step kernels' memory traffic, comments
    aside: their source (mrt_kernels.hip up to the adjoint section: helpers,
    ghost and step kernels), their launchers, the headers they include, and
    the population layout (the layout functions of mrt_api.hip)."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_1004_5442_amd", "csrc")
    with open(os.path.join(csrc, "mrt_kernels.hip")) as fh:
        text = fh.read()
    head = text[:text.index("// ---------------------------------------------------------------- adjoint")]
    launchers = []
    for name in ("hipError_t launch_step(", "hipError_t launch_step2("):
        i0 = text.index(name)
        launchers.append(text[i0:text.index("\n}\n", i0)])
    with open(os.path.join(csrc, "mrt_api.hip")) as fh:
        api = fh.read()
    layout = api[api.index("// Population layout"):api.index("bool bc_ok(")]
    h = hashlib.sha256()
    for part in [head, *launchers, layout]:
        h.update(hashlib.sha256(_code_only(part).encode()).digest())
    for name in STEP_HEADERS:
        with open(os.path.join(csrc, name)) as fh:
            h.update(hashlib.sha256(_code_only(fh.read()).encode()).digest())
    return h.hexdigest()


def measured_traffic(precision, per_pass, band_rows):
    """HBM bytes per two-step-kernel launch (counter readings scaled by the
    copy calibration), or None when they do not describe the kernel that
    runs."""
    m = MEASURED_TRAFFIC
    if (precision != "fp32_eq64" or per_pass != 2 or m["digest"] != kernel_digest()
            or band_rows != m["band_rows"]):
        return None
    gib_kib = 1024.0 * 1024.0
    fetch = m["fetch_kib"] * gib_kib / m["fetch_copy_kib"]
    write = m["write_kib"] * gib_kib / m["write_copy_kib"]
    return int(round((fetch + write) * 1024))


def _events_time(stream, fn, nsteps):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn(nsteps)
    e1.record(stream)
    e1.synchronize()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


# The GPU reaches its sustained-load clocks only after ~60-100 ms of
# continuous work (measured on the headline grid: two-step passes take
# 0.62-0.66 ms right after a short start, settle at 0.567 ms after ~100
# passes, and slow down again after 2 s idle).  Each measurement therefore
# first keeps the GPU busy for PREHEAT_S with the same kernels on a scratch
# copy of the workload (a second instance, configured the same way and then
# freed), so that the measured instance runs exactly the requested warm-up
# steps from its initial state and the timed region exactly the requested
# steps, at the clocks a sustained run holds.
PREHEAT_S = 0.3


def _preheat(step, min_s=PREHEAT_S, max_steps=None):
    """Step a scratch instance in chunks of 16 steps for at least min_s
    seconds, but not past max_steps (the workload's own run length: some
    shock tubes of the batch break down a thousand steps after it, in the
    oracle too); returns the steps run."""
    import torch
    ran = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < min_s and (max_steps is None or ran + 16 <= max_steps):
        step(16)
        ran += 16
        torch.cuda.synchronize()
    return ran


def _configured_solver(case, precision, autotune, tile_rows, scheme, per_pass):
    from paper_1004_5442_amd.solver import solver_for_case
    s = solver_for_case(case, precision)
    if scheme:
        s.set_scheme(**scheme)
    if per_pass == 2:
        s.set_steps_per_pass(2, tile_rows)
    elif tile_rows:
        s.set_steps_per_pass(1, 0)
        s.set_tile(tile_rows)
    elif autotune:
        s.autotune(4)
    return s


def time_solver(case, precision, steps, warmup, autotune=True, tile_rows=0, scheme=None,
                per_pass=0):
    """per_pass 1 or 2 with tile_rows: that kernel and band height; else the
    autotuner's choice (autotune) or the library's default."""
    import torch
    s = _configured_solver(case, precision, autotune, tile_rows, scheme, per_pass)
    heat = _configured_solver(case, precision, False, tile_rows, scheme, per_pass)
    if autotune and not tile_rows and not per_pass:
        heat.set_tile(*s.tile())
        k, r = s.steps_per_pass()
        if not scheme:
            heat.set_steps_per_pass(k, r if k == 2 else 0)
    pre = _preheat(heat.step, max_steps=case.nsteps)
    heat.close()
    del heat
    s.step(warmup)
    s.prepare(steps)        # capture the step graphs outside the timed region
    s.sync()
    sec = _events_time(torch.cuda.current_stream(), s.step, steps)
    s.sync()      # raises if the run went unhealthy
    tile = s.tile()
    pp = s.steps_per_pass()
    s.close()
    mlups = case.cells * steps / sec / 1e6
    return {"mlups": mlups, "sec": sec, "ms_per_step": 1e3 * sec / steps, "tile": tile,
            "per_pass": pp[0], "band_rows": pp[1], "preheat_steps": pre}


def time_batch(steps, warmup, precision="fp32_eq64"):
    """The batched form: 512 seeded shock tubes (nx 200..4000, ny 4), FP32
    populations with FP64 collision (or the given precision), graph-captured
    passes in the launch the batch autotuner picks (the tube march, four
    steps per pass, on this batch); the step counts are rounded up to whole
    passes."""
    import torch

    from paper_1004_5442_amd import workloads as W
    from paper_1004_5442_amd.batch import Batch
    cases = W.tube_batch(512, seed=0)
    b = Batch(cases, precision)
    b.autotune(4)
    heat = Batch(cases, precision)
    heat.set_tile(*b.tile())
    k, r = b.steps_per_pass()
    heat.set_steps_per_pass(k, r if k == 2 else 0)
    pre = _preheat(heat.step, max_steps=cases[0].nsteps)
    heat.close()
    del heat
    steps, warmup = -(-steps // k) * k, -(-warmup // k) * k
    b.step(warmup)
    b.prepare(steps)
    torch.cuda.synchronize()
    sec = _events_time(torch.cuda.current_stream(), b.step, steps)
    b.moments(0)              # raises if any instance went unhealthy
    cells = b.cells
    tile = b.tile()
    pp = b.steps_per_pass()
    b.close()
    return {"mlups": round(cells * steps / sec / 1e6, 1), "cells": cells, "instances": len(cases),
            "ms_per_step": round(1e3 * sec / steps, 4), "steps": steps, "tile_rows": tile[0],
            "kernel": {1: "step_kernel", 2: "step2_kernel", 4: "tube_kernel"}[pp[0]],
            "steps_per_pass": pp[0], "band_rows": pp[1], "preheat_steps": pre,
            "roofline_frac": round(cells * BYTES_PER_SITE[precision] * steps / sec / 1e9 / HBM_PEAK_GBS, 4)}


def time_adjoint_large(n, steps):
    """Adjoint step vs forward step on an n^2 periodic grid of the adjoint
    workload's kind (FP32 storage, FP64 collision), large enough to leave the
    caches: the adjoint moves 192 B per site (lam read, f read, lam write)."""
    import torch

    from paper_1004_5442_amd import workloads as W
    from paper_1004_5442_amd.solver import Solver
    case, _ = W.adjoint_problem(n=n, seed=0, nsteps=10)
    sv = Solver(n, n, "fp32_eq64")
    # the 256^2 workload's Courant numbers: dt shrinks with the cell size
    sv.set_params(case.gamma, case.s, case.dt * 256 / n, case.dx, case.dy)
    rho0 = torch.tensor(case.rho, device="cuda")
    T0 = torch.tensor(case.T, device="cuda")
    zero = torch.zeros_like(rho0)
    f, g = sv.empty_state(), sv.empty_state()
    sv.init_buffer(rho0, zero, zero, T0, f)
    lam, lam2 = sv.empty_state(), sv.empty_state()
    sv.init_buffer(rho0, zero, zero, T0, lam)
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")

    def fwd(k):
        for _ in range(k):
            sv.step_buffers(f, g)

    def adj(k):
        for _ in range(k):
            sv.adjoint_step(lam, f, lam2, ds)

    fwd(3)
    adj(3)
    _preheat(fwd)     # repeated launches on the same input: f is not advanced
    st = torch.cuda.current_stream()
    t_f = _events_time(st, fwd, steps) / steps
    t_a = _events_time(st, adj, steps) / steps
    sv.close()
    return {"grid": f"{n}x{n}", "adjoint_step_ms": round(1e3 * t_a, 4), "forward_step_ms": round(1e3 * t_f, 4),
            "adjoint_over_forward": round(t_a / t_f, 3), "adjoint_mlups": round(n * n / t_a / 1e6, 1),
            "adjoint_roofline_frac": round(n * n * 192 / t_a / 1e9 / HBM_PEAK_GBS, 4)}


def time_adjoint(steps):
    """Adjoint step vs forward step on the 256^2 periodic adjoint workload
    (FP32 storage, FP64 collision), and one full gradient (500-step forward,
    sqrt(N) checkpoints, backward) vs the plain 500-step forward (each the
    median of five runs)."""
    import torch

    from paper_1004_5442_amd import workloads as W
    from paper_1004_5442_amd.adjoint import density_after
    from paper_1004_5442_amd.solver import Solver
    case, T_target = W.adjoint_problem(n=256, seed=0, nsteps=500)
    n = case.nx
    sv = Solver(n, n, "fp32_eq64")
    sv.set_params(case.gamma, case.s, case.dt, case.dx, case.dy)
    rho0 = torch.tensor(case.rho, device="cuda")
    T0 = torch.tensor(case.T, device="cuda")
    zero = torch.zeros_like(rho0)
    f, g = sv.empty_state(), sv.empty_state()
    sv.init_buffer(rho0, zero, zero, T0, f)
    lam, lam2 = sv.empty_state(), sv.empty_state()
    sv.init_buffer(rho0, zero, zero, T0, lam)
    ds = torch.zeros(16, dtype=torch.float64, device="cuda")

    def fwd(k):
        for _ in range(k):
            sv.step_buffers(f, g)

    def adj(k):
        for _ in range(k):
            sv.adjoint_step(lam, f, lam2, ds)

    fwd(5)
    adj(5)
    _preheat(fwd)     # repeated launches on the same input: f is not advanced
    st = torch.cuda.current_stream()
    t_f = _events_time(st, fwd, steps) / steps
    t_a = _events_time(st, adj, steps) / steps
    args = (case.gamma, case.dt, case.dx, case.dy, case.nsteps)
    s0 = torch.tensor(case.s, device="cuda")
    with torch.no_grad():
        target = density_after(rho0, torch.tensor(T_target, device="cuda"), s0, sv, *args)
    def fwd_full():
        with torch.no_grad():
            density_after(rho0, T0, s0, sv, *args)
        torch.cuda.synchronize()

    def grad():
        r = rho0.clone().requires_grad_(True)
        L = 0.5 * ((density_after(r, T0, s0, sv, *args) - target) ** 2).sum()
        L.backward()
        torch.cuda.synchronize()

    def median_s(fn, reps=5):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t0)
        return sorted(ts)[reps // 2]

    torch.cuda.synchronize()
    t_fwd_full = median_s(fwd_full)
    grad()          # the first backward also starts autograd's device threads
    t_grad = median_s(grad)
    sv.close()
    return {"grid": f"{n}x{n}", "adjoint_step_ms": round(1e3 * t_a, 4), "forward_step_ms": round(1e3 * t_f, 4),
            "adjoint_over_forward": round(t_a / t_f, 3),
            "adjoint_mlups": round(n * n / t_a / 1e6, 1),
            "adjoint_roofline_frac": round(n * n * 192 / t_a / 1e9 / HBM_PEAK_GBS, 4),
            "gradient_500_steps_s": round(t_grad, 4), "forward_500_steps_s": round(t_fwd_full, 4),
            "gradient_over_forward": round(t_grad / t_fwd_full, 3),
            "note": "256^2 FP32 fits the Infinity Cache: effective, not HBM, bandwidth"}


def roofline(case, precision, r, traffic=None):
    """Algorithmic bytes of one step-kernel launch (bytes per site update x
    the site updates of one launch: cells x steps per pass) over the
    event-timed launch (which also holds the ~5 us reflecting-wall ghost
    launch: achieved is a slight underestimate of the kernel's own rate)."""
    per_pass = r.get("per_pass", 1)
    per_launch_bytes = BYTES_PER_SITE[precision] * case.cells * per_pass
    achieved = per_launch_bytes / (r["sec"] / r["steps"] * per_pass) / 1e9
    out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
           "traffic_unit": "bytes per launch", "algorithmic_bytes": per_launch_bytes,
           "kernel": "step2_kernel" if per_pass == 2 else "step_kernel",
           "bytes_per_site": BYTES_PER_SITE[precision], "site_updates_per_launch": case.cells * per_pass}
    if traffic is not None:
        # what the launch really moves, per second (counter readings)
        out["traffic_GBs"] = round(traffic / (r["sec"] / r["steps"] * per_pass) / 1e9, 1)
    if per_pass == 2:
        out["note"] = ("two time steps per launch: each launch reads f^n once and writes f^{n+2}, so "
                       "its HBM traffic (traffic_GBs) is about 0.61 x the per-step algorithmic bytes; "
                       "that traffic moves at ~4.6-4.7 TB/s, near the 4.7-5.3 TB/s that plain "
                       "streaming reaches on this chip, with the vector ALUs ~58 % busy")
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_band(rows, steps, start_barrier=None, out=None):
    """The FP64 oracle (one BLAS thread) on a 4096 x rows band of the
    headline workload: `steps` steps after setup; returns (cells x steps,
    start, end) in wall-clock seconds.  With a barrier every worker starts
    its timed steps together."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import mrt
    from paper_1004_5442_amd import workloads as W
    case = W.shock_bubble(n=4096, ny=rows)
    bcmap = {"periodic": 0, "eq": 1, "outflow": 2, "reflect": 3}
    p = mrt.Params(gamma=case.gamma, s=case.s, dt=case.dt, dx=case.dx, dy=case.dy,
                   bc=[bcmap[b] for b in case.bc], side_state=case.side_state)
    with threadpool_limits(limits=1):
        f = mrt.init_populations(case.rho, case.ux, case.uy, case.T, p)
        if start_barrier is not None:
            start_barrier.wait()
        t0 = time.time()
        for _ in range(steps):
            f = mrt.step(f, p)
        t1 = time.time()
    assert np.isfinite(f).all()
    res = (case.cells * steps, t0, t1)
    if out is not None:
        out.put(res)
    return res


def cpu_baseline(rows1=1024, steps1=6, rows_all=256, steps_all=6, max_workers=16):
    """The FP64 NumPy oracle on the host cores, as it stands: one process on
    a 4096 x rows1 band, then one process per core (capped at the CPU share
    a one-GPU host gives a job, max_workers) each on its own 4096 x rows_all
    band, started together; MLUPS = site updates / wall time."""
    import multiprocessing as mp
    n1, t0, t1 = _oracle_band(rows1, steps1)
    v1 = n1 / (t1 - t0) / 1e6
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    workers = max(1, min(max_workers, avail))
    ctx = mp.get_context("spawn")        # fresh interpreters: no GPU state inherited
    bar = ctx.Barrier(workers)
    q = ctx.Queue()
    procs = [ctx.Process(target=_oracle_band, args=(rows_all, steps_all, bar, q)) for _ in range(workers)]
    for pr in procs:
        pr.start()
    res = [q.get(timeout=600) for _ in procs]
    for pr in procs:
        pr.join()
    total = sum(r[0] for r in res)
    wall = max(r[2] for r in res) - min(r[1] for r in res)
    vall = total / wall / 1e6
    return {"value": round(vall, 4), "unit": "MLUPS", "cores": workers, "kind": "oracle",
            "value_1core": round(v1, 4), "value_allcore": round(vall, 4),
            "nproc": os.cpu_count(), "cores_available": avail, "cpu_model": _cpu_model(),
            "sample": (f"FP64 NumPy oracle (one BLAS thread per process) on bands of the 4096^2 "
                       f"shock-bubble case: 1 core {steps1} steps of 4096x{rows1}; all cores "
                       f"{workers} processes x {steps_all} steps of 4096x{rows_all} each, "
                       f"started together")}


def extra_legs(head, prec, steps):
    """The extra measurements, by name (each a function returning its JSON
    object); `bench.py --only NAME` runs one of them alone (for profiling)."""
    from paper_1004_5442_amd import workloads as W
    k = max(20, steps // 4)
    k += k & 1

    def device_copy():
        # the practical streaming ceiling: a plain 1 GiB device-to-device
        # copy (read + write of 1 GiB each), after the same 0.3 s preheat
        import torch
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        _preheat(lambda n: [b.copy_(a) for _ in range(n)])
        n = 20
        sec = _events_time(torch.cuda.current_stream(), lambda m: [b.copy_(a) for _ in range(m)], n)
        gbs = 2 * (1 << 30) * n / sec / 1e9
        del a, b
        return {"GBs": round(gbs, 1), "fraction_of_peak": round(gbs / HBM_PEAK_GBS, 4),
                "note": "plain 1 GiB device copy (torch copy_), 2 GiB moved per copy: the rate "
                        "a pure stream reaches on this box"}

    def one_step():
        r1 = time_solver(head, prec, k, 3, tile_rows=HEADLINE_TILE_ROWS, per_pass=1)
        r1["steps"] = k
        return {"mlups": round(r1["mlups"], 1), "band_rows": HEADLINE_TILE_ROWS,
                "roofline_frac": roofline(head, prec, r1)["frac"]}

    def fp64():
        # the library's default at this size: two steps per pass, 64-row bands
        r64 = time_solver(head, "fp64", k, 3, tile_rows=FP64_BAND_ROWS, per_pass=2)
        r64["steps"] = k
        return {"mlups": round(r64["mlups"], 1), "steps_per_pass": 2, "band_rows": FP64_BAND_ROWS,
                "roofline_frac": roofline(head, "fp64", r64)["frac"]}

    def fp64_one_step():
        r64 = time_solver(head, "fp64", k, 3, tile_rows=HEADLINE_TILE_ROWS)
        r64["steps"] = k
        return {"mlups": round(r64["mlups"], 1), "band_rows": HEADLINE_TILE_ROWS,
                "roofline_frac": roofline(head, "fp64", r64)["frac"]}

    def fp32():
        r32 = time_solver(head, "fp32", k, 3, tile_rows=HEADLINE_BAND_ROWS, per_pass=2)
        r32["steps"] = k
        return {"mlups": round(r32["mlups"], 1), "steps_per_pass": 2,
                "roofline_frac": roofline(head, "fp32", r32)["frac"]}

    def riemann(pr):
        def run():
            rp = W.riemann2d(n=1024, seed=0)
            rr = time_solver(rp, pr, 2 * k, 5)
            rr["steps"] = 2 * k
            return {"mlups": round(rr["mlups"], 1), "steps_per_pass": rr["per_pass"],
                    "effective_GBs": roofline(rp, pr, rr)["achieved"],
                    "note": "fits the 256 MB Infinity Cache: effective, not HBM, bandwidth"}
        return run

    def stripe():
        # one GPU's share of the headline grid in the stripe decomposition at
        # eight GPUs (4096 x 512 rows of the same workload; 134 MB per state:
        # cache-resident), in the autotuner's launch; the halo exchange that
        # would replace the reflecting ghost pass is not modelled
        c = W.shock_bubble(n=4096, ny=512)
        rr = time_solver(c, prec, 2 * k, 5)
        rr["steps"] = 2 * k
        return {"mlups": round(rr["mlups"], 1), "steps_per_pass": rr["per_pass"],
                "band_rows": rr["band_rows"], "effective_GBs": roofline(c, prec, rr)["achieved"],
                "note": "4096 x 512: one GPU's share at eight; fits the 256 MB Infinity Cache"}

    def variants():
        out = {}
        for name, sch, bps in (("split", {"split": True}, 256), ("lw_cross", {"lw_cross": True}, 128),
                               ("split_lw_cross", {"split": True, "lw_cross": True}, 256)):
            rv = time_solver(head, prec, k, 3, autotune=False, scheme=sch)
            out[name] = {"mlups": round(rv["mlups"], 1), "bytes_per_site": bps,
                         "roofline_frac": round(bps * rv["mlups"] * 1e6 / 1e9 / HBM_PEAK_GBS, 4)}
        return out

    def rm(pr):
        def run():
            rr = time_solver(W.rm_instability(), pr, 4 * k, 64)
            rr["steps"] = 4 * k
            return {"mlups": round(rr["mlups"], 1), "ms_per_step": round(rr["ms_per_step"], 5),
                    "tile_rows": rr["tile"][0], "steps_per_pass": rr["per_pass"],
                    "note": "36,000 cells: launch-latency bound (captured graphs of 64 steps)"}
        return run

    def paper_riemann2d():
        # section (c)'s own problem at its printed size (500^2, FP64 MRT):
        # cache-resident, effective bandwidth
        c = W.paper_riemann2d()
        rr = time_solver(c, "fp64", 4 * k, 5)
        rr["steps"] = 4 * k
        return {"mlups": round(rr["mlups"], 1), "steps_per_pass": rr["per_pass"],
                "effective_GBs": roofline(c, "fp64", rr)["achieved"],
                "note": "fits the 256 MB Infinity Cache: effective, not HBM, bandwidth"}

    def strong_shock():
        # section (b)'s strong-shock tube (1100 x 1, FP64 MRT, dt = 1e-6):
        # launch-latency bound
        c = W.strong_shock_tube(1.4, False)
        rr = time_solver(c, "fp64", 16 * k, 64)
        return {"mlups": round(rr["mlups"], 1), "ms_per_step": round(rr["ms_per_step"], 5),
                "steps_per_pass": rr["per_pass"],
                "steps_for_t_0.13_s": round(c.nsteps * rr["ms_per_step"] / 1e3, 3),
                "note": "1,100 cells: launch-latency bound (captured graphs of 64 passes; the "
                        "autotuner's steps per pass, 4 = the tube march)"}

    return {
        "device_copy_1gib": device_copy,
        "fp32_eq64_one_step_per_pass": one_step,
        "fp64_same_grid": fp64,
        "fp64_one_step_per_pass": fp64_one_step,
        "fp32_same_grid": fp32,
        "stripe_4096x512_fp32_eq64": stripe,
        "riemann2d_1024_fp32_eq64": riemann("fp32_eq64"),
        "riemann2d_1024_fp64": riemann("fp64"),
        "scheme_variants_4096_fp32_eq64": variants,
        "rm_instability_360x100_fp32_eq64": rm("fp32_eq64"),
        "rm_instability_360x100_fp64": rm("fp64"),
        "paper_riemann2d_500_fp64": paper_riemann2d,
        "strong_shock_tube_1100_fp64": strong_shock,
        "batched_512_tubes": lambda: time_batch(max(50, steps // 2), 5),
        "batched_512_tubes_fp64": lambda: time_batch(max(50, steps // 2), 5, "fp64"),
        "adjoint_256": lambda: time_adjoint(100),
        "adjoint_2048": lambda: time_adjoint_large(2048, 20),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--steps-per-pass", type=int, default=HEADLINE_PER_PASS, choices=(1, 2),
                    help="kernel of the headline run: two time steps per pass or one")
    ap.add_argument("--rows", type=int, default=0,
                    help="band height of the headline run (default: 32 for two steps per "
                         "pass, 8 for one)")
    ap.add_argument("--only", default=None,
                    help="run only this extra measurement (a key of 'extra') and print its "
                         "JSON object: for profiling one kernel")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is described in the design notes but not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1004_5442_amd import workloads as W
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    n = 4096
    head = W.shock_bubble(n=n)
    prec = "fp32_eq64"
    if args.only:
        legs = extra_legs(head, prec, args.steps)
        if args.only not in legs:
            sys.exit(f"--only: one of {sorted(legs)}")
        print(json.dumps({"leg": args.only, **legs[args.only]()}), flush=True)
        return
    rows = args.rows or (HEADLINE_BAND_ROWS if args.steps_per_pass == 2 else HEADLINE_TILE_ROWS)
    r = time_solver(head, prec, args.steps, args.warmup, tile_rows=rows, per_pass=args.steps_per_pass)
    r["steps"] = args.steps
    out = {
        "metric": "MLUPS (million lattice-site updates per second) of the MRT FD-LB step",
        "value": round(r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "preheat_s": PREHEAT_S,
        "preheat_steps": r["preheat_steps"],
        "ms_per_step": round(r["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 storage, f64 collision",
        "data": "synthetic",
        "config": {"workload": f"shock_bubble {n}x{n} (Mach-5 shock on a density-3 bubble, "
                               f"gamma 1.4, Pr 0.71, reflect/inflow/outflow)",
                   "cells": head.cells, "precision": prec, "steps_per_pass": r["per_pass"],
                   "band_rows": r["band_rows"]},
        "roofline": roofline(head, prec, r, measured_traffic(prec, r["per_pass"], r["band_rows"])),
    }
    if not args.no_extra:
        out["extra"] = {name: fn() for name, fn in extra_legs(head, prec, args.steps).items()}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
