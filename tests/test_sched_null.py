"""The serving loop's scheduler core (queue, tickets, admission of pooled
ray slots / images / latents, the coarse-to-fine tick table, completion,
failure and cancellation) on a null device, on the CPU, built with
ThreadSanitizer: DIST_EBUSY when the queue is full, DIST_ENOTFOUND for
unknown or already-read tickets, DIST_ECANCELLED at shutdown, DIST_EHIP for
every job running across a failed tick, DIST_ENUMERIC for a job the device
flags, injected allocation failures, and
exclusive ownership of every image slot and ray-slot range."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "sched", "null_sched.cpp")


@pytest.fixture(scope="module")
def binary(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("sched") / "null_sched")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=thread", "-pthread",
           "-I", os.path.join(ROOT, "paper_1911_13225_amd", "csrc"), "-I", os.path.join(ROOT, "include"),
           SRC, "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    return out


@pytest.mark.parametrize("scenario", ["mixed", "busy", "cancel", "tickfail", "numeric"])
def test_scheduler_core_on_a_null_device(binary, scenario):
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66 second_deadlock_stack=1")
    r = subprocess.run([binary, scenario], capture_output=True, text=True, timeout=240, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-6000:]
    assert r.returncode == 0, (r.returncode, r.stdout, r.stderr[-4000:])
    assert f"ok {scenario}" in r.stdout
