"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only; the device code is built as usual).

The sources are built once more with the sanitizers on the host side only
(each -fsanitize flag behind -Xarch_host), and the host-side test files
(transforms, equilibrium, collision and cell adjoint on the host, header
exports, every argument check of the C ABI) run against that build in a
child process with the sanitizer runtime preloaded.  Any report fails the
test."""
import glob
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1004_5442_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


@pytest.fixture(scope="module")
def sanitized_library():
    rt = _runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or the clang sanitizer runtime is not available")
    out = os.path.join(tempfile.mkdtemp(prefix="mrtlb_asan_"), "libmrtlb.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
           os.path.join(CSRC, "mrt_kernels.hip"), os.path.join(CSRC, "mrt_api.hip"), "-o", out]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-3000:]
    return out, rt


def test_host_code_is_clean_under_sanitizers(sanitized_library):
    lib, rt = sanitized_library
    env = dict(os.environ, MRTLB_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    probe = subprocess.run([sys.executable, "-c", "import paper_1004_5442_amd.lib as L; print(L.LIB_PATH)"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stdout + probe.stderr
    tests = [os.path.join(ROOT, "tests", f) for f in ("test_host_library.py", "test_host_validation.py")]
    res = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p",
                          "no:cacheprovider", *tests], cwd=ROOT, env=env, capture_output=True,
                         text=True, timeout=900)
    report = res.stdout[-4000:] + res.stderr[-4000:]
    print(report)
    assert res.returncode == 0, report
    assert "AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, report
    assert " passed" in res.stdout
