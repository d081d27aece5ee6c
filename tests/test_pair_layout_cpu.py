"""Host check of the two-wave tile fragment layouts (no GPU).

tests/cpp/test_pair_layout.cpp emulates v_mfma_f32_16x16x4_f32 and
v_mfma_f32_16x16x32_{bf16,f16} with their lane layouts over the fragments that
layout_pair_f32 / layout_pair_16 write for each member of a pair, feeding the
member's own defect registers and then its partner's as B the way the kernel does,
and checks x = K d on every lane for H = 16..128. Built with ROCm's clang++ as host
code (factor.cpp needs _Float16)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang++" if os.path.exists("/opt/rocm/llvm/bin/clang++") \
    else shutil.which("clang++")


@pytest.mark.skipif(CLANG is None, reason="clang++ not available")
def test_pair_fragment_layouts_emulated(tmp_path):
    exe = str(tmp_path / "pair_layout")
    csrc = os.path.join(ROOT, "paper_2608_25666_amd", "csrc")
    subprocess.run([CLANG, "-std=c++17", "-O1", "-I", csrc,
                    os.path.join(ROOT, "tests", "cpp", "test_pair_layout.cpp"),
                    os.path.join(csrc, "factor.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    print(r.stdout[-800:])
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok")
