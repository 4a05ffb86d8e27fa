"""Host AddressSanitizer + UndefinedBehaviorSanitizer build of libpotato's
host code: tests/abi_sanitize_main.cpp calls every entry point along its
argument-checking paths and creates a context, so that out-of-bounds
accesses or undefined arithmetic in the host code abort the run.  The
sanitizers instrument host code only (each -fsanitize= follows
-Xarch_host); no kernel is launched.  Skipped when hipcc or the sanitizer
runtimes are missing."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2308_12698_amd", "csrc")


@pytest.mark.timeout(600)
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "abi_sanitize"
    sources = [os.path.join(CSRC, f) for f in ("kernels.hip", "collide.hip", "abi.hip", "pipeline.hip")]
    cmd = [hipcc, "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"), *sources, os.path.join(HERE, "abi_sanitize_main.cpp"),
           "-lrocprofiler-sdk-roctx", "-o", str(exe)]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=540)
    # only a missing sanitizer runtime skips (the output names the build's
    # own files, so a bare "asan" would also match a compile error)
    err = (build.stderr or "").lower()
    if build.returncode != 0 and "clang_rt" in err and ("not found" in err or "no such file" in err):
        pytest.skip("sanitizer runtime not available: " + build.stderr[-300:])
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ)
    # the HIP runtime keeps allocations for the process lifetime: leaks are not ours to judge
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    run = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    out = run.stdout + run.stderr
    assert run.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
    assert "abi sanitizer run: ok" in out
