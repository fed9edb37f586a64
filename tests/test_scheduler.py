"""The replanning server's scheduler (allocator, FIFO admission under slot and
memory limits, quantum slicing, deadlines, cancellation, latency percentiles),
built for the host with g++ and driven by a mock executor; a copy built with
AddressSanitizer and UndefinedBehaviorSanitizer runs the same checks."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "test_sched.cpp")


@pytest.mark.parametrize("flags", [["-O2"], ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover"]])
def test_scheduler_core(tmp_path, flags):
    exe = str(tmp_path / "test_sched")
    subprocess.run(["g++", "-std=c++17", "-Wall", "-Werror", *flags, SRC, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sched OK" in r.stdout
