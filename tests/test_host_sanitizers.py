"""The host side of the C ABI built with AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the device code is compiled as
usual) and run without a GPU: argument validation for every width class,
drive and wall, workspace layouts, and the failure paths of lb_create that
return before any device call."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_runtime_under_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = tmp_path / "host_sanitized"
    csrc = os.path.join(ROOT, "paper_1310_7450_amd", "csrc")
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "lb_runtime.hip"), os.path.join(csrc, "lb_kernels.hip"),
           os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"), "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert build.returncode == 0, build.stderr[-2000:]
    # the HIP runtime library keeps its own allocations until exit: no leak report
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr[-2000:]
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr[-2000:]
