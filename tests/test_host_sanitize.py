"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host_sanitize/driver.cpp drives validation (every supported grid, and invalid grids and
options, which must be refused with CHAN_EINVAL and leave *out untouched), the FP64 operator
precompute of every supported N (closed and open channel, two Reynolds numbers: every entry
finite, and the influence-matrix homogeneous solutions on their Dirichlet rows to 1e-14 of their
coefficient magnitude, which pins the tau solve's boundary-row refinement), the seeded
initial condition and the plane-pass tiling candidates.  The library sources are compiled as
usual for gfx950, with the sanitizers on the host side only; no device code runs (there is no
GPU here, and every device path stops at its first HIP call)."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2301_09889_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["kernels.hip", "plane_pass.hip", "column_pass.hip", "env.cpp", "precompute.cpp", "initial.cpp"]
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-sanitize-recover=all"]
FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC] + SANITIZE


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + FLAGS + ["-c", src, "-o", obj], capture_output=True, text=True)
        return obj, r

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, srcs))
    for (obj, r), src in zip(results, srcs):
        assert r.returncode == 0, f"{src}:\n{r.stderr[-3000:]}"
    exe = str(tmp_path / "driver")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + SANITIZE + [o for o, _ in results] + ["-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ)
    # the HIP runtime keeps allocations until exit: leak reports would be its, not ours
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "host checks passed" in r.stdout, (r.stdout[-2000:], r.stderr[-5000:])
