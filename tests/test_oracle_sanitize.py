"""The C breadth-first oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, on the CPU) and driven over 400 small
seeded instances with NaN / infinite values, positions outside the grid,
no particles, unit dimensions, particle rates, forward-only coupling,
duplicate, inadmissible and out-of-range seeds: any out-of-bounds access,
leak or undefined behaviour aborts the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run(
        ["gcc", "-O1", "-g", "-std=c99", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-o", exe, os.path.join(ROOT, "tests", "oracle_sanitize_main.c"),
         os.path.join(ROOT, "oracle", "grow_bfs.c"), "-lm"],
        capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("no sanitizer runtime")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "0 failures" in run.stdout
