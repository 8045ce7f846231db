"""Host sanitizer builds (CPU only), under AddressSanitizer and
UndefinedBehaviorSanitizer: the oracle driven through every entry point on
small, ragged and degenerate inputs (tests/sanitize/oracle_driver.c), and the
request server's host-side scheduling driven by a fake executor
(tests/sanitize/sched_driver.cpp)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _build_and_run(src, out, extra):
    gcc = shutil.which("gcc")
    if not gcc:
        pytest.skip("gcc not available")
    cmd = [gcc, "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *extra, src, "-o", out, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    # verify_asan_link_order=0: the environment may preload a library of its
    # own ahead of the sanitizer runtime; leak checking needs ptrace, which a
    # sandbox may deny, so it is off (the driver frees what it allocates)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([out], capture_output=True, text=True, env=env, timeout=300)


def test_oracle_under_asan_and_ubsan(tmp_path):
    r = _build_and_run(os.path.join(HERE, "sanitize", "oracle_driver.c"),
                       str(tmp_path / "oracle_driver"), [])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "all calls returned" in r.stdout


def _build_and_run_cpp(src, out, extra):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", *extra, src, "-o", out]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([out], capture_output=True, text=True, env=env, timeout=300)


def test_server_scheduler_with_fake_executor_under_asan_and_ubsan(tmp_path):
    """The request server's host-side scheduling state (ks_sched.h: first-fit
    arena, budget-bounded segment pool, first-come-first-served admission)
    against a brute-force allocator model and a simulated executor
    (tests/sanitize/sched_driver.cpp), under the sanitizers."""
    csrc = os.path.join(os.path.dirname(HERE), "paper_1511_07207_amd", "csrc")
    r = _build_and_run_cpp(os.path.join(HERE, "sanitize", "sched_driver.cpp"),
                           str(tmp_path / "sched_driver"), ["-I", csrc])
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr
    assert "scheduler checks passed" in r.stdout
