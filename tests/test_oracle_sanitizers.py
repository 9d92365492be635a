"""The FP64 oracle's C source under AddressSanitizer and
UndefinedBehaviorSanitizer (host only): a driver runs 2D and 3D rollouts and
backward passes with floor contact, a clamp and three kinds of obstacle for
every loss kind; any out-of-bounds access, leak or undefined behaviour ends the
run with a report. Built serially and with OpenMP (three threads)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("openmp", [False, True])
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path, openmp):
    exe = str(tmp_path / "oracle_driver")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off"] + (["-fopenmp"] if openmp else []) + [
           f"-I{ORACLE}", "-o", exe, os.path.join(HERE, "oracle_sanitize_driver.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "sanitizer" in (r.stderr or "").lower() and "cannot find" in (r.stderr or ""):
        pytest.skip("sanitizer runtime not installed: " + r.stderr[-200:])
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="3")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.strip() == "ok", (run.stdout[-500:], run.stderr[-3000:])
