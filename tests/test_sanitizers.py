"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU, gcc).

tests/native/oracle_sanitize.c drives the oracle over small systems (one and two OpenMP
threads, the factor export, a non-SPD input, rejected arguments) and checks its results;
built with -fsanitize=address,undefined and -fno-sanitize-recover, any out-of-bounds
access, leak or undefined operation ends the run with a non-zero status."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-fopenmp",
           os.path.join(ROOT, "oracle", "bmpc_oracle.c"),
           os.path.join(ROOT, "tests", "native", "oracle_sanitize.c"), "-lm", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip() == "ok"
