"""Host code under sanitizers (host compilers only, no GPU):
* the planner (plan.cpp) with AddressSanitizer and UndefinedBehaviorSanitizer
  over many lattice shapes, leaf edges, partitions and periodic flags
  (tests/native/plan_check.cpp): every plan's invariants hold and invalid
  inputs are refused;
* the request server (serve.cpp: queueing, HBM admission, batch forming, the
  slot threads, cancel / wait / release) with ThreadSanitizer and with
  AddressSanitizer + UndefinedBehaviorSanitizer (tests/native/serve_check.cpp),
  its device layer replaced by host code through tests/native/stub: several
  threads submit concurrently and every finished result is checked bit for bit.
No memory error, data race or undefined behaviour may be reported."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_planner_under_asan_ubsan(tmp_path):
    exe = tmp_path / "plan_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
           os.path.join(ROOT, "paper_1102_3137_amd", "csrc", "plan.cpp"), "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "0 failures" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr


SERVE_SOURCES = [os.path.join(ROOT, "tests", "native", "serve_check.cpp"),
                 os.path.join(ROOT, "paper_1102_3137_amd", "csrc", "serve.cpp"),
                 os.path.join(ROOT, "paper_1102_3137_amd", "csrc", "plan.cpp")]
STUB = os.path.join(ROOT, "tests", "native", "stub")


def _clang():
    """A clang++ with the ThreadSanitizer runtime (the ROCm toolchain's, or one
    on PATH); GCC 11's runtime does not intercept pthread_cond_clockwait,
    which std::condition_variable::wait_for uses, and then reports false
    races."""
    for c in [os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "llvm", "bin", "clang++"),
              shutil.which("clang++")]:
        if c and os.path.exists(c):
            return c
    return None


def _run_serve_check(exe, env):
    run = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    print(run.stdout)
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "0 failures" in run.stdout
    return run


@pytest.mark.skipif(_clang() is None, reason="needs clang++ with the TSan runtime")
def test_server_under_tsan(tmp_path):
    exe = tmp_path / "serve_tsan"
    cmd = [_clang(), "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread", "-I", STUB,
           *SERVE_SOURCES, "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    run = _run_serve_check(exe, dict(os.environ, TSAN_OPTIONS="halt_on_error=1"))
    assert "WARNING: ThreadSanitizer" not in run.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_server_under_asan_ubsan(tmp_path):
    exe = tmp_path / "serve_asan"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-pthread",
           "-I", STUB, *SERVE_SOURCES, "-o", str(exe)]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr
    run = _run_serve_check(exe, dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                                     UBSAN_OPTIONS="print_stacktrace=1"))
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
