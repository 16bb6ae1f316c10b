"""CPU unit test of the request server's scheduler (ch_sched.hpp): the C++
driver in tests/native/sched_test.cpp runs it with a fake executor and a
fake clock, built with ThreadSanitizer (and separately with
AddressSanitizer), so data races and memory errors in the host-side
scheduling fail the test. No GPU involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_test.cpp")


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not installed")
    exe = str(tmp_path / "sched_test")
    subprocess.check_call([gxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-pthread",
                           "-I", os.path.join(ROOT, "paper_2209_12310_amd", "csrc"),
                           "-I", os.path.join(ROOT, "include"), SRC, "-o", exe])
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1",
               ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="halt_on_error=1")
    p = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert p.returncode == 0, p.stderr[-4000:]
    assert p.stdout.strip() == "ok"
