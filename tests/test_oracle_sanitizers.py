"""Host AddressSanitizer + UndefinedBehaviorSanitizer build of the FP64
reference: every entry point runs on small ragged inputs
(tests/oracle_sanitize_main.cpp) and any out-of-bounds access or undefined
arithmetic aborts the run.  CPU only; skipped when g++ or the sanitizer
runtimes are missing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(300)
def test_oracle_under_asan_and_ubsan(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "oracle_sanitize"
    cmd = [gxx, "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", os.path.join(HERE, "oracle_sanitize_main.cpp"), "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True)
    if build.returncode != 0 and "asan" in (build.stderr or "").lower():
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "2"
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=240)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
    assert "oracle sanitizer run: ok" in out
