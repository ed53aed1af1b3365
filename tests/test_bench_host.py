"""The benchmark's host-side parts on the CPU: the CPU-baseline leg (the
oracle on one core and on every core, with the host's description), the
one-GPU guard, and the traffic digest that keeps stale counter readings out
of the roofline object."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_cpu_baseline_reports_one_core_and_all_cores():
    out = bench.cpu_baseline(rows1=8, steps1=1, rows_all=4, steps_all=1, max_workers=2)
    for key in ("value", "value_1core", "value_allcore", "cores", "nproc", "cores_available",
                "cpu_model", "sample", "unit", "kind"):
        assert key in out, key
    assert out["kind"] == "oracle" and out["unit"] == "MLUPS"
    assert 1 <= out["cores"] <= 2 and out["value"] == out["value_allcore"]
    assert out["value_1core"] > 0 and out["value_allcore"] > 0
    json.dumps(out)


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode != 0 and "one GPU" in res.stderr


def test_traffic_reading_is_tied_to_the_kernel_sources():
    """The stored counter readings apply only to the kernel they were taken
    on: the current sources' digest, the headline precision, two steps per
    pass and the band height; anything else reports no traffic."""
    assert bench.measured_traffic("fp32_eq64", 2, bench.HEADLINE_BAND_ROWS) is not None
    assert bench.measured_traffic("fp32_eq64", 1, bench.HEADLINE_BAND_ROWS) is None
    assert bench.measured_traffic("fp64", 2, bench.HEADLINE_BAND_ROWS) is None
    assert bench.measured_traffic("fp32_eq64", 2, 16) is None
    saved = dict(bench.MEASURED_TRAFFIC)
    try:
        bench.MEASURED_TRAFFIC["digest"] = "0" * 64
        assert bench.measured_traffic("fp32_eq64", 2, bench.HEADLINE_BAND_ROWS) is None
    finally:
        bench.MEASURED_TRAFFIC.update(saved)
