"""The FP64 oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
on the host (gcc), running every mode it has (body force with and without
the flow-induced density, one-row channels, the half-link and Zou-He moving
walls, the time-integrated stress, the pressure drive, the stress force) for
a few steps: no memory error, no undefined behaviour, finite populations and,
where the method conserves it, the mass to round-off."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_sanitized"
    cmd = ["gcc", "-g", "-O1", "-std=c11", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "lb_oracle.c"),
           os.path.join(ROOT, "oracle", "sanitize_driver.c"), "-o", str(exe), "-lm"]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("the sanitizer runtime is not installed: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "ERROR" not in run.stderr and "runtime error" not in run.stderr, run.stderr
