"""Host check of the printed-iteration kernel's FP64 fragment layout (no GPU).

tests/cpp/test_literal_layout.cpp emulates v_mfma_f64_16x16x4_f64 with the lane
layout measured on gfx950 (accumulator item e of lane group g holds row g + 4e; the
FP32 instruction uses 4g + e) over the fragments layout_f64 writes, feeding each
lane's own right-hand-side registers as the B operand the way the kernel does, and
checks x = K r + k v0 on every lane for H = 2..128 (projection and printed-iteration
factors). Built with ROCm's clang++ as host code: factor.cpp needs _Float16.
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") \
    else shutil.which("clang++")


@pytest.mark.skipif(CLANG is None, reason="clang++ not available")
def test_fp64_fragment_layout_emulated(tmp_path):
    exe = str(tmp_path / "literal_layout")
    csrc = os.path.join(ROOT, "paper_2608_25666_amd", "csrc")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-I", csrc,
                    os.path.join(ROOT, "tests", "cpp", "test_literal_layout.cpp"),
                    os.path.join(csrc, "factor.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout[-600:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
