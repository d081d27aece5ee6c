"""Build libprism_proj.so (HIP for gfx950) in-tree.

    python -m paper_2608_25666_amd.build [--jobs N] [--incremental]

Every HIP/C++ source under csrc/ is compiled with hipcc for gfx950 (objects in
_build/ at the repository root) and linked into paper_2608_25666_amd/libprism_proj.so.
Packed FP32 instructions are disabled for all device code.
"""

from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(ROOT, "_build", "obj")
LIB = os.path.join(PKG, "libprism_proj.so")
ARCH = "gfx950"

COMMON = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # MFMA accumulators in VGPRs rather than AGPRs: the tile loops read every product
    # with VALU instructions, and the AGPR form adds a v_accvgpr_read per register
    # (H = 100 FP32 inner loop 1197 -> 1168 instructions, 393 -> 377 registers)
    "-mllvm", "-amdgpu-mfma-vgpr-form=1",
    "-I", INCLUDE, "-I", CSRC,
]


def hipcc() -> str:
    for cand in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


_INCLUDE_RE = re.compile(r'^\s*#\s*include\s+"([^"]+)"', re.M)


def _newest_input(src: str) -> float:
    """Newest modification time of src and the local headers it includes, recursively."""
    seen, todo, newest = set(), [src], 0.0
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        newest = max(newest, os.path.getmtime(f))
        with open(f, encoding="utf-8") as fh:
            for name in _INCLUDE_RE.findall(fh.read()):
                for d in (os.path.dirname(f), CSRC, INCLUDE):
                    cand = os.path.join(d, name)
                    if os.path.exists(cand):
                        todo.append(cand)
                        break
    return newest


def _compile(src: str, incremental: bool):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj) and os.path.getmtime(obj) > _newest_input(src):
        return obj, 0.0, ""
    cmd = [hipcc()] + COMMON + ["-x", "hip", "-c", src, "-o", obj]
    t0 = time.time()
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{err}")
    return obj, time.time() - t0, err


def build(jobs: int = 0, incremental: bool = False, verbose: bool = False) -> str:
    """Compile every source and link the shared library; returns its path."""
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = jobs or max(1, min(16, os.cpu_count() or 4))
    srcs = sources()
    objs = []
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, incremental): s for s in srcs}
        for f in cf.as_completed(futs):
            obj, dt, err = f.result()
            objs.append(obj)
            if verbose:
                print(f"  {os.path.basename(futs[f]):24s} {dt:6.1f} s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + sorted(objs)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, LIB)
    build_abi_consumer(verbose)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f} s", flush=True)
    return LIB


ABI_DEMO_SRC = os.path.join(os.path.dirname(PKG), "tests", "cpp", "abi_solve.cpp")
ABI_DEMO = os.path.join(os.path.dirname(PKG), "tests", "cpp", "abi_solve")


def build_abi_consumer(verbose: bool = False):
    """The native C-ABI consumer used by the tests (host program linking the library)."""
    if not os.path.exists(ABI_DEMO_SRC):
        return None
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-O2", "-std=c++17", "-I", INCLUDE, ABI_DEMO_SRC,
           "-L", PKG, "-lprism_proj", f"-Wl,-rpath,{PKG}", "-Wl,-rpath,$ORIGIN/../../paper_2608_25666_amd",
           "-o", ABI_DEMO]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building {ABI_DEMO_SRC} failed:\n{r.stderr}")
    if verbose:
        print(f"built {ABI_DEMO}", flush=True)
    return ABI_DEMO


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--jobs", type=int, default=0)
    ap.add_argument("--incremental", action="store_true")
    a = ap.parse_args(argv)
    build(jobs=a.jobs, incremental=a.incremental, verbose=True)


if __name__ == "__main__":
    main(sys.argv[1:])
