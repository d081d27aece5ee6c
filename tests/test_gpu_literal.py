"""The printed Bregman iteration on the GPU (prism_proj_literal) against the oracle's
oracle.admm.literal_joint: same inputs (the FP32 samples widened to FP64), same
number of passes, FP64 arithmetic on both sides.

The two evaluate the same map with different FP64 rounding: the GPU applies a
precomputed inverse on the matrix cores, forms the G^T terms with prefix sums and
takes Step 3 through its exact closed form lambda' = (lambda + x' - x~) / 2 (pinned in
the oracle tests); the oracle LU-solves the saddle system with the dense G and
evaluates Step 3 as printed, which multiplies the solve's rounding by delta G^T G.
Both are accurate to about kappa * 2^-52 * |x| per pass, kappa = cond(I + delta G^T G)
<= 1 + 32 delta / dt^4 (the jerk rows' weight times ||D2||^2 <= 16): 5e6 at dt = 0.05,
2e8 at dt = 0.02. Bars, with L passes and X = max |x|:
  |x_gpu - x_oracle| <= 2^-24 |x| + L * 2^-52 * kappa * X + 1e-12   (FP32 rounding of
                        the result plus the FP64 drift of L passes),
  |viol_gpu - viol_oracle| <= 4 (L * 2^-52 * kappa * X + 1e-12) / dt^2 + 1e-9 |viol|
                        (a velocity error moves a jerk row by up to 4 / dt^2 times it).
"""

import numpy as np
import pytest

from oracle import admm, problem
import workloads as W
from workloads import recipes as WC

pytestmark = pytest.mark.gpu


def _run_gpu(req, iters, delta, x_init=None, inplace=False):
    import torch
    from paper_2608_25666_amd import Projector
    P = Projector(req.H, req.nj, req.dt, req.bounds, 1.0, weights="default")
    x = torch.from_numpy(req.samples).cuda()
    xi = None if x_init is None else torch.from_numpy(x_init).cuda()
    out = x if inplace else None
    o, viol = P.literal(x, req.q0, req.v0, iters, delta=delta, x_init=xi, out=out)
    torch.cuda.synchronize()
    res = o.cpu().numpy(), viol.cpu().numpy()
    P.close()
    return res


def _run_oracle(req, iters, delta, x_init=None):
    N, H, nj = req.samples.shape
    X = np.empty((N, H, nj))
    V = np.empty((N, nj))
    for j in range(nj):
        lim = problem.joint_limits(req.bounds, j)
        xi = None if x_init is None else x_init[:, :, j].astype(np.float64)
        xj, vj = admm.literal_joint(req.samples[:, :, j].astype(np.float64), H, req.dt, lim,
                                    float(req.q0[j]), float(req.v0[j]), delta=delta,
                                    iters=iters, x_init=xi)
        X[:, :, j] = xj
        V[:, j] = vj
    return X, V


def _check(req, xg, vg, xo, vo, label, iters, delta):
    kappa = 1.0 + 32.0 * delta / req.dt ** 4
    drift = iters * 2.0 ** -52 * kappa * np.abs(xo).max() + 1e-12
    ex = np.abs(xg - xo)
    bar = 2.0 ** -24 * np.abs(xo) + drift
    ev = np.abs(vg - vo)
    vbar = 4.0 * drift / req.dt ** 2 + 1e-9 * np.abs(vo)
    print(f"{label}: x max-abs {ex.max():.3e} (FP64 drift bar {drift:.1e}), violation max-abs "
          f"{ev.max():.3e} (bar {vbar.min():.1e}+), oracle violation max {vo.max():.3e}")
    assert np.all(ex <= bar), np.unravel_index(np.argmax(ex - bar), ex.shape)
    assert np.all(ev <= vbar), np.unravel_index(np.argmax(ev - vbar), ev.shape)


CASES = [
    # seed, N, H, nj, dt, passes, delta, sample kind
    (1, 37, 50, 12, 0.05, 20, 1.0, "smooth"),    # 3 tiles per joint, ragged tail
    (2, 16, 13, 3, 0.05, 1, 1.0, "white"),       # one pass, one full tile
    (3, 33, 5, 2, 0.05, 50, 1.0, "white"),       # H = 5: last two lane groups past the horizon
    (4, 20, 100, 2, 0.02, 20, 0.3, "smooth"),    # long horizon, small dt
    (5, 17, 128, 1, 0.05, 10, 1.0, "smooth"),    # largest horizon
    (6, 5, 2, 1, 0.1, 5, 1.0, "white"),          # smallest horizon
    (7, 40, 31, 4, 0.05, 15, 2.0, "white"),      # H not a multiple of 4
    (8, 24, 69, 3, 0.02, 12, 1.0, "smooth"),     # odd chunk length (18)
]


@pytest.mark.parametrize("case", CASES, ids=[f"H{c[2]}_N{c[1]}_J{c[3]}_L{c[5]}" for c in CASES])
def test_literal_matches_oracle(case):
    seed, N, H, nj, dt, iters, delta, kind = case
    req = WC.make_request(seed, N=N, H=H, nj=nj, dt=dt, kind=kind)
    xg, vg = _run_gpu(req, iters, delta)
    xo, vo = _run_oracle(req, iters, delta)
    _check(req, xg, vg, xo, vo, f"H={H} N={N} nj={nj} passes={iters}", iters, delta)


def test_literal_zero_passes_and_zero_start():
    """Zero passes return the first iterate with x_1 = v0; a zero first iterate (the
    x0 = 0 start) matches the oracle started from zeros."""
    req = WC.make_request(11, N=21, H=50, nj=3, dt=0.05, kind="white")
    xg, vg = _run_gpu(req, 0, 1.0)
    want = req.samples.astype(np.float64).copy()
    want[:, 0, :] = req.v0[None, :]
    np.testing.assert_array_equal(xg, want.astype(np.float32))
    xo, vo = _run_oracle(req, 0, 1.0)
    _check(req, xg, vg, xo, vo, "zero passes", 0, 1.0)
    z = np.zeros_like(req.samples)
    xg, vg = _run_gpu(req, 20, 1.0, x_init=z)
    xo, vo = _run_oracle(req, 20, 1.0, x_init=z)
    _check(req, xg, vg, xo, vo, "x0 = 0, 20 passes", 20, 1.0)


def test_literal_in_place_equals_out_of_place():
    req = WC.make_request(12, N=50, H=20, nj=6, dt=0.05, kind="white")
    a, va = _run_gpu(req, 15, 1.0)
    b, vb = _run_gpu(req, 15, 1.0, inplace=True)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(va, vb)


def test_literal_benchmark_workload():
    """The launch the benchmark times: N = 2048, H = 50, 12 joints, dt = 0.02, 20
    passes, delta = 1, every output compared."""
    req = WC.mpc_batch(0)
    xg, vg = _run_gpu(req, 20, 1.0)
    xo, vo = _run_oracle(req, 20, 1.0)
    _check(req, xg, vg, xo, vo, "N=2048 H=50 nj=12 passes=20", 20, 1.0)


def test_literal_errors_and_empty():
    import torch
    from paper_2608_25666_amd import PrismError, Projector
    req = WC.make_request(13, N=8, H=20, nj=2, dt=0.05, kind="white")
    P = Projector(req.H, req.nj, req.dt, req.bounds, 1.0, weights="default")
    x = torch.from_numpy(req.samples).cuda()
    for bad in (dict(delta=0.0), dict(delta=-1.0), dict(delta=float("nan")), dict(iters=-1)):
        kw = dict(iters=5, delta=1.0)
        kw.update(bad)
        with pytest.raises(PrismError):
            P.literal(x, req.q0, req.v0, kw["iters"], delta=kw["delta"])
    with pytest.raises(PrismError):
        P.literal(x, req.q0, np.full(2, 99.0), 5)          # v0 outside the velocity bounds
    empty = torch.zeros((0, 20, 2), dtype=torch.float32, device="cuda")
    o, v = P.literal(empty, req.q0, req.v0, 5)
    torch.cuda.synchronize()
    assert o.shape == (0, 20, 2) and v.shape == (0, 2)
    P.close()


def test_literal_very_large_batch_sampled():
    """131072 samples x 12 joints (98304 tiles), 10 passes: sampled outputs against the
    oracle run on those samples alone (columns are independent)."""
    import torch
    from paper_2608_25666_amd import Projector
    req = WC.make_request(53, N=131072, H=20, nj=12, dt=0.05, kind="white")
    P = Projector(req.H, req.nj, req.dt, req.bounds, 1.0, weights="default")
    x = torch.from_numpy(req.samples).cuda()
    o, viol = P.literal(x, req.q0, req.v0, 10, delta=1.0)
    torch.cuda.synchronize()
    pick = np.r_[0, 1, 65535, 65536, 131070, 131071]
    xg, vg = o.cpu().numpy()[pick], viol.cpu().numpy()[pick]
    P.close()
    sub = WC.Request(H=req.H, nj=req.nj, dt=req.dt, bounds=req.bounds, q0=req.q0, v0=req.v0,
                     samples=np.ascontiguousarray(req.samples[pick]), rho=1.0, iters=10, name="")
    xo, vo = _run_oracle(sub, 10, 1.0)
    _check(sub, xg, vg, xo, vo, "131072 x 12, sampled", 10, 1.0)
