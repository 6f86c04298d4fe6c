"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source is compiled with the sanitizers on its host side only (device
code is built as usual and never launched), linked with
tests/host_sanitize/driver.cpp, and run on the CPU: argument checks of every
entry point, workspace sizing, the persistent-batch planner, the Step 2
configuration code (Section 3.2), the internal parameters and the Step 4
extraction.  Leak checking is off: the HIP runtime keeps allocations for the
life of the process."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2305_04318_amd.build import SOURCES  # every source of the library

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_04318_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
FLAGS = ["-std=c++17", "-O1", "-g", "--offload-arch=gfx950",
         "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
         "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-value",
         "-I", os.path.join(ROOT, "include")]


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    srcs.append(os.path.join(ROOT, "tests", "host_sanitize", "driver.cpp"))

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + FLAGS + ["-c", src, "-o", obj], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_driver")
    r = subprocess.run([HIPCC] + FLAGS + objs + ["-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # the sanitizers are really linked in
    syms = subprocess.run(["nm", exe], capture_output=True, text=True).stdout
    assert "__asan_init" in syms and "__ubsan_handle" in syms
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-6000:]
    assert "host checks passed" in out
    assert "AddressSanitizer" not in out and "runtime error" not in out
