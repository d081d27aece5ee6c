"""The C ABI driven by a native program (tests/cpp/abi_solve.cpp, built by
__graft_entry__.build()): no Python or PyTorch between the caller and the
library. Its projection matches the FP64 oracle at the FP32 bar and its FP64
feasibility report matches the oracle's loop-based violations."""

import os
import subprocess

import numpy as np
import pytest

from oracle import admm, feasibility
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "cpp", "abi_solve")


def _write(path, r, iters, weights, alpha, tol, precision=0, mode=0):
    H, nj, N = r.H, r.nj, r.N
    with open(path, "wb") as f:
        np.array([H, nj, N, iters, precision, mode], dtype=np.int32).tofile(f)
        np.array([r.dt, r.rho], dtype=np.float64).tofile(f)
        np.array(weights, dtype=np.float64).tofile(f)
        np.array([alpha, tol], dtype=np.float32).tofile(f)
        np.array([np.broadcast_to(np.asarray(v, np.float64), (nj,)) for v in r.bounds.as_list()],
                 dtype=np.float64).tofile(f)
        np.asarray(r.q0, np.float64).tofile(f)
        np.asarray(r.v0, np.float64).tofile(f)
        np.ascontiguousarray(r.samples, dtype=np.float32).tofile(f)


def _read(path, N, H, nj):
    with open(path, "rb") as f:
        x = np.fromfile(f, np.float32, N * H * nj).reshape(N, H, nj)
        rp = np.fromfile(f, np.float32, N * nj).reshape(N, nj)
        rd = np.fromfile(f, np.float32, N * nj).reshape(N, nj)
        it = np.fromfile(f, np.int32, N * nj).reshape(N, nj)
        v = np.fromfile(f, np.float64, N * nj * 5).reshape(N, nj, 5)
    return x, rp, rd, it, v


@pytest.mark.skipif(not os.path.exists(EXE), reason="native consumer not built")
def test_native_consumer_matches_oracle(tmp_path):
    r = W.make_request(61, N=40, H=24, nj=3, dt=0.05, kind="white")
    w = (1.0, 2.5 / 24, 4.0, 20.0)
    src, dst = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(src, r, 90, w, 1.6, 0.0)
    p = subprocess.run([EXE, src, dst], capture_output=True, text=True, timeout=120)
    print(p.stdout, p.stderr)
    assert p.returncode == 0
    x, rp, rd, it, v = _read(dst, r.N, r.H, r.nj)
    O = admm.solve_request(r.samples, r.H, r.dt, r.bounds, r.q0, r.v0, iters=90, alpha=1.6,
                           weights=w)
    err = np.abs(x - O.x).max()
    print(f"native C-ABI consumer: max-abs vs oracle {err:.3e}")
    assert err <= 1e-4
    np.testing.assert_allclose(rp, O.r_p, atol=1e-4, rtol=1e-3)
    assert np.all(it == 90)
    V = feasibility.violations(x, r.dt, r.bounds, r.q0, r.v0)
    for k, name in enumerate(("pos", "vel", "acc", "jerk", "eq")):
        np.testing.assert_allclose(v[..., k], V[name], atol=1e-9, rtol=1e-9)


@pytest.mark.skipif(not os.path.exists(EXE), reason="native consumer not built")
@pytest.mark.parametrize("alpha", [1.0, 1.6])
def test_native_consumer_plain_signatures(tmp_path, alpha):
    """prism_proj_create (scalar penalty) and prism_proj_solve (handle options set with
    prism_proj_set_options) from C: the projection after a fixed count equals the
    oracle's at the FP32 bar; the FP64 feasibility report equals the oracle's."""
    r = W.make_request(62, N=37, H=31, nj=2, dt=0.05, kind="white")
    src, dst = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(src, r, 120, (1.0, 1.0, 1.0, 1.0), alpha, 0.0, mode=1)
    p = subprocess.run([EXE, src, dst], capture_output=True, text=True, timeout=120)
    print(p.stdout, p.stderr)
    assert p.returncode == 0
    x, rp, rd, it, v = _read(dst, r.N, r.H, r.nj)
    assert np.all(it == -1)                   # the plain solve reports no counts
    O = admm.solve_request(r.samples, r.H, r.dt, r.bounds, r.q0, r.v0, iters=120, alpha=alpha)
    err = np.abs(x - O.x).max()
    print(f"plain signatures alpha {alpha}: max-abs {err:.3e}")
    assert err <= 1e-4
    np.testing.assert_allclose(rp, O.r_p, atol=1e-4, rtol=1e-3)
    V = feasibility.violations(x, r.dt, r.bounds, r.q0, r.v0)
    for k, name in enumerate(("pos", "vel", "acc", "jerk", "eq")):
        np.testing.assert_allclose(v[..., k], V[name], atol=1e-9, rtol=1e-9)
