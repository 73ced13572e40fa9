"""Race and memory checks of the serving scheduler core on the CPU: the
stress driver tests/sched_stress.cpp runs several client threads against the
scheduler (fake backend, moving memory budget, failures, oversized
requests) under ThreadSanitizer and under AddressSanitizer + UBSan."""
import os
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sched_stress.cpp")


# ThreadSanitizer needs a runtime that intercepts pthread_cond_clockwait
# (condition_variable::wait_for on a steady clock): the ROCm LLVM clang has
# one; gcc 11's does not and reports a false "double lock".
CLANG = "/opt/rocm/llvm/bin/clang++"


def build_and_run(flags, tmp):
    exe = os.path.join(tmp, "stress")
    cxx = CLANG if os.path.exists(CLANG) else "g++"
    cmd = [cxx, "-std=c++17", "-O1", "-g", "-pthread"] + flags + [SRC, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "sanitizer" in r.stderr.lower() and "cannot find" in r.stderr.lower():
            pytest.skip("sanitizer runtime not installed")
        raise AssertionError(r.stderr)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)


@pytest.mark.parametrize("flags", [["-fsanitize=thread"],
                                   ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"]],
                         ids=["tsan", "asan_ubsan"])
def test_scheduler_under_sanitizer(flags):
    with tempfile.TemporaryDirectory() as tmp:
        r = build_and_run(flags, tmp)
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, r.stdout + r.stderr[-4000:]
    assert "errors 0" in r.stdout
