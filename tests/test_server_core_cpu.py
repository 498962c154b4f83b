"""Host-only check of the serving layer's scheduling core (device-memory arena
and admission policy) with a fake executor; no GPU is involved.

The C++ driver (server_core_check.cpp) includes the same header the server is
built from and checks, over random robots, submissions and completion delays:
first-fit arena accounting and coalescing; at most one request in flight per
robot; per-robot FIFO order; the oldest idle heads admitted first; max_slots,
max_batch and the budget respected; every request served once arrivals stop.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_scheduling_core_with_fake_executor(tmp_path):
    exe = str(tmp_path / "server_core_check")
    cmd = ["g++", "-std=c++17", "-O1", "-Wall", "-Wextra", "-Werror",
           "-I", os.path.join(ROOT, "paper_2504_06437_amd", "csrc"),
           os.path.join(ROOT, "tests", "server_core_check.cpp"), "-o", exe,
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip().endswith("OK"), r.stdout + r.stderr
