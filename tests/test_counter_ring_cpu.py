"""The rule by which solves reuse a handle's tile-queue counter sets
(paper_2608_25666_amd/csrc/counter_ring.h), built with g++ and checked in a
discrete-event model of streams and launches, without a GPU."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_counter_ring_never_shares_a_set(tmp_path):
    exe = str(tmp_path / "test_counter_ring")
    src = os.path.join(ROOT, "tests", "cpp", "test_counter_ring.cpp")
    inc = os.path.join(ROOT, "paper_2608_25666_amd", "csrc")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-I", inc, src, "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
