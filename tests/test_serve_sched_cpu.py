"""The projection server's admission scheduler (pool allocator, FIFO admission,
per-controller serialisation, LRU eviction of idle warm state), built with g++
and exercised without a GPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_host_checks(tmp_path):
    exe = str(tmp_path / "test_serve_sched")
    src = os.path.join(ROOT, "tests", "cpp", "test_serve_sched.cpp")
    inc = os.path.join(ROOT, "paper_2608_25666_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-I", inc, src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
