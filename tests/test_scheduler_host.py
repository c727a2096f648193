"""The serving scheduler on the CPU, driven by a fake executor.

The scheduler (admission by device-memory budget, strict FIFO, bounded
queue, slot choice, retirement) is host-only code shared by the HIP server;
tests/sched_harness.cpp runs it against a simulated device: forced
allocation failures, a slow device that fills the queue, failed launches and
jobs that fail on the device, and a long randomised stream of all of them.  Built with g++, once plainly and once with the
address and undefined-behaviour sanitizers (host code only).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched_harness.cpp")
SCENARIOS = ["fifo", "alloc_failure", "slow_device", "failures", "slots", "random"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


@pytest.fixture(scope="module", params=["plain", "sanitized"])
def harness(request, tmp_path_factory):
    out = str(tmp_path_factory.mktemp("sched") / f"sched_{request.param}")
    flags = ["-std=c++17", "-O1", "-Wall", "-Werror", f"-I{ROOT}"]
    if request.param == "sanitized":
        flags += ["-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-fno-sanitize-recover=all"]
    proc = subprocess.run(["g++", *flags, SRC, "-o", out], capture_output=True, text=True)
    assert proc.returncode == 0, proc.stderr
    return out


@pytest.mark.parametrize("scenario", SCENARIOS)
def test_scheduler_scenario(harness, scenario):
    proc = subprocess.run([harness, scenario], capture_output=True, text=True, timeout=60)
    assert proc.returncode == 0, proc.stdout + proc.stderr
    assert proc.stdout.strip() == f"ok {scenario}"
