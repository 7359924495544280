"""The C++ oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/host/oracle_sanitize.cpp drives every integration path of
oracle/kerr_oracle.cpp on small inputs (camera rays with crossing records and
constants on two threads, RK4, coordinate time with dense output and t_end
landing, a recorded trajectory, a controller trace, the Boyer-Lindquist map and
both fixed-step charts).  Built with g++ and both sanitizers (host code only),
any out-of-bounds access, leak or undefined arithmetic aborts the run.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(ROOT, "oracle", "kerr_oracle.cpp"), os.path.join(HERE, "host", "oracle_sanitize.cpp")]


def test_oracle_clean_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    build = subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
                            "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", *SRCS,
                            "-pthread", "-o", exe], capture_output=True, text=True)
    if build.returncode != 0 and "asan" in build.stderr.lower() and "cannot find" in build.stderr.lower():
        pytest.skip("g++ has no sanitizer runtime here")
    assert build.returncode == 0, build.stderr
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "runtime error" not in run.stderr, run.stderr
    assert "all paths ran" in run.stdout
