"""The serving layer's admission control (paper_1604_07893_amd/csrc/hp_sched.h:
arrival-order admission under a slot cap and an HBM budget, first-fit
placement with a coalescing free list), compiled for the CPU with g++ and
exercised by tests/host/sched_check.cpp with a fake executor (each request
finishes after its own number of loops): placement and coalescing cases,
head-of-line blocking, the error paths of the serving step (hp::serve_step:
a failed set-up, a failed rerun set-up, a loop that fails after finishing
some requests, a successful rerun), and 20 random replays of 400 requests checking the
slot cap, the budget, disjoint placements, arrival order, completion and a
fully coalesced arena at the end. No GPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_admission_control(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "sched_check"
    subprocess.run([gxx, "-std=c++17", "-O1", "-Wall", "-I",
                    os.path.join(ROOT, "paper_1604_07893_amd", "csrc"),
                    os.path.join(ROOT, "tests", "host", "sched_check.cpp"), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
