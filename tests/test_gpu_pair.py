"""GPU parity of the two-wave tile kernel (options tile_waves = 2): a tile's steps are
split over a pair of waves that hand over sums, boundary terms and defects through LDS.
Same iteration as the one-wave kernel in another summation order, so it is held to the
same bars against the FP64 oracle: FP32 1e-4 at equal counts; reduced forms at their
fixed-count and residual-mode bars (tests/test_gpu_forms.py; FP16 at a fixed count
below against the one-wave kernel's own error on the same request); residual-mode stops
checked as in tests/stops.py."""

import numpy as np
import pytest

from oracle import admm
import workloads as W

pytestmark = pytest.mark.gpu

TOL_BF16_TAIL = 2e-2
# FP16 GEMM operands, 100 iterations with the last 10 in FP32, on the H = 50 smooth request
# below: the one-wave kernel itself measures 7.5e-4 (alpha 1) and 7.1e-4 (alpha 1.8) there
# (its 5e-4 bar in tests/test_gpu_forms.py was set on other requests: the drift from FP16
# rounding of d depends on the request's contraction history). The pair rounds the same d
# values, so it is held to 1e-3 and to no more than 5% above the one-wave kernel's error.
TOL_F16_FIXED = 1e-3
TOL_REDUCED_RESIDUAL = 4e-3


def _solve(r, iters, opts, weights="default", samples=None):
    import torch
    from paper_2608_25666_amd import Projector
    P = Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights=weights)
    s = r.samples if samples is None else samples
    x = torch.from_numpy(np.ascontiguousarray(s)).cuda()
    it = torch.zeros((x.shape[0], r.nj), dtype=torch.int32, device="cuda")
    out, rp, rd = P.solve(x, r.q0, r.v0, iters, opts=opts, iters_out=it)
    torch.cuda.synchronize()
    res = out.cpu().numpy(), rp.cpu().numpy(), rd.cpu().numpy(), it.cpu().numpy(), P.weights
    P.close()
    return res


@pytest.mark.parametrize("H,N,nj,dt,kind", [
    (20, 37, 3, 0.05, "white"),     # chunks of 3, padding in the last two chunks
    (17, 16, 2, 0.05, "white"),     # H = 17: chunk 7 holds one step
    (24, 50, 2, 0.02, "smooth"),    # exact fit
    (50, 40, 12, 0.02, "smooth"),   # chunks of 7, six padding steps
    (56, 33, 2, 0.05, "white"),     # exact fit
    (100, 35, 3, 0.02, "smooth"),   # chunks of 13
    (97, 18, 2, 0.05, "white"),     # chunk 7 holds one step
])
@pytest.mark.parametrize("alpha", [1.0, 1.8])
def test_pair_fixed_count_matches_oracle(H, N, nj, dt, kind, alpha):
    from paper_2608_25666_amd import options
    r = W.make_request(90 + H, N=N, H=H, nj=nj, dt=dt, kind=kind)
    x, rp, rd, it, w = _solve(r, 120, options(alpha=alpha, tile_waves=2))
    O = admm.solve_request(r.samples, H, dt, r.bounds, r.q0, r.v0, iters=120, alpha=alpha,
                           weights=w)
    err = np.abs(x - O.x).max()
    print(f"H={H} N={N} nj={nj} alpha={alpha}: max-abs {err:.2e}; r_p {np.abs(rp - O.r_p).max():.1e}")
    assert err <= 1e-4
    assert np.all(it == 120)
    np.testing.assert_allclose(rp, O.r_p, atol=1e-4, rtol=1e-3)
    np.testing.assert_allclose(rd, O.r_d, atol=3e-4, rtol=1e-3)


@pytest.mark.parametrize("alpha", [1.0, 1.8])
@pytest.mark.parametrize("prec,tol", [("fp16", TOL_F16_FIXED), ("bf16", TOL_BF16_TAIL)])
def test_pair_reduced_forms_fixed_count(prec, tol, alpha):
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP16
    p = PREC_BF16 if prec == "bf16" else PREC_FP16
    r = W.make_request(95, N=48, H=50, nj=4, dt=0.02, kind="smooth")
    xs = []
    for tw in (1, 2):
        x, rp, rd, it, w = _solve(r, 100, options(precision=p, fp32_tail=10, alpha=alpha,
                                                  tile_waves=tw))
        xs.append(x)
    O = admm.solve_request(r.samples, r.H, r.dt, r.bounds, r.q0, r.v0, iters=100, alpha=alpha,
                           weights=w)
    errs = [float(np.abs(x - O.x).max()) for x in xs]
    print(f"{prec}+10 fixed 100, alpha {alpha}: max-abs one-wave {errs[0]:.2e}, pair {errs[1]:.2e}")
    assert errs[1] <= tol
    assert errs[1] <= 1.05 * errs[0] + 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_pair_mpc_batch_residual_mode(prec):
    """The 2048 x 12 x H = 50 batch at the benchmark settings with two-wave tiles: every
    column at residual <= 1e-3; sampled tiles against the oracle run to their counts."""
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP16, PREC_FP32
    from stops import check_residual_mode
    p = {"fp32": PREC_FP32, "fp16": PREC_FP16, "bf16": PREC_BF16}[prec]
    r = W.mpc_batch()
    o = options(precision=p, alpha=1.8, tol=1e-3, fp32_tail=0 if prec == "fp32" else 10,
                tile_waves=2)
    x, rp, rd, it, w = _solve(r, 20000, o)
    assert np.all(np.maximum(rp, rd) <= 1e-3)
    pick = np.r_[np.arange(0, 32), np.arange(2016, 2048)]
    joints = sorted({int(np.argmax(it.max(axis=0))), 0, 6})
    check_residual_mode(x[pick], rp[pick], rd[pick], it[pick], pick, r.samples, r.H, r.dt,
                        r.bounds, r.q0, r.v0, tol=1e-3, check_every=10, cap=20000, alpha=1.8,
                        weights=w, xbar=1e-4 if prec == "fp32" else TOL_REDUCED_RESIDUAL,
                        check_stops=prec == "fp32", label=f"pair mpc {prec}", joints=joints)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_pair_long_horizon_residual_mode(prec):
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP32
    from stops import check_residual_mode
    p = PREC_FP32 if prec == "fp32" else PREC_BF16
    r = W.long_horizon_batch()
    o = options(precision=p, alpha=1.8, tol=1e-3, fp32_tail=0 if prec == "fp32" else 10,
                tile_waves=2)
    x, rp, rd, it, w = _solve(r, 20000, o)
    assert np.all(np.maximum(rp, rd) <= 1e-3)
    rows = np.r_[np.arange(0, 16), np.arange(8176, 8192)]
    joints = sorted({int(np.argmax(it.max(axis=0))), 3})
    check_residual_mode(x[rows], rp[rows], rd[rows], it[rows], rows, r.samples, r.H, r.dt,
                        r.bounds, r.q0, r.v0, tol=1e-3, check_every=10, cap=20000, alpha=1.8,
                        weights=w, xbar=1e-4 if prec == "fp32" else TOL_REDUCED_RESIDUAL,
                        check_stops=prec == "fp32", label=f"pair long {prec}", joints=joints)


def test_pair_iteration_counts_track_the_one_wave_kernel():
    """Same iteration, different summation order: residual-mode stop counts of the two
    kernels agree for most tiles and differ by at most one check period otherwise."""
    from paper_2608_25666_amd import options
    r = W.make_request(96, N=256, H=50, nj=6, dt=0.02, kind="smooth")
    kw = dict(alpha=1.8, tol=1e-3)
    _, _, _, it1, _ = _solve(r, 20000, options(tile_waves=1, **kw))
    _, _, _, it2, _ = _solve(r, 20000, options(tile_waves=2, **kw))
    d = np.abs(it1 - it2)
    print(f"equal counts {np.mean(d == 0):.2f}, max difference {d.max()}")
    assert np.all(d <= 10)
    assert np.mean(d == 0) >= 0.8


def test_pair_feasible_input_and_nan():
    """A feasible sample with x~_1 = v0 comes back unchanged bit for bit (every defect is
    zero, alpha = 1); a NaN sample gives NaN residuals for its column only."""
    import torch
    from oracle import feasibility
    from paper_2608_25666_amd import Projector, options
    H, nj, N, dt = 50, 3, 32, 0.05
    t = np.arange(1, H + 1) * dt
    base = np.stack([0.2 * np.sin(2 * np.pi * 0.4 * t + p) for p in (0.0, 0.7, 1.9)], axis=1)
    samples = np.repeat(base[None], N, axis=0).astype(np.float32)
    samples += np.linspace(-0.02, 0.02, N, dtype=np.float32)[:, None, None]
    v0 = samples[0, 0, :].astype(np.float64)
    samples[:, 0, :] = samples[0, 0, :]
    bounds = W.UR5E_BIMANUAL_BOUNDS(nj)
    q0 = np.zeros(nj)
    viol = feasibility.max_violation(samples.astype(np.float64), dt, bounds, q0, v0)
    assert max(viol.values()) == 0.0
    bad = samples.copy()
    bad[5, 17, 1] = np.nan
    P = Projector(H, nj, dt, bounds, 1.0, weights="default")
    for arr, nan in ((samples, False), (bad, True)):
        x = torch.from_numpy(arr).cuda()
        out, rp, rd = P.solve(x, q0, v0, 60, opts=options(tile_waves=2))
        torch.cuda.synchronize()
        o, rpn = out.cpu().numpy(), rp.cpu().numpy()
        if not nan:
            np.testing.assert_array_equal(o, samples)
            assert np.all(rpn == 0.0) and np.all(rd.cpu().numpy() == 0.0)
        else:
            keep = np.ones((N, nj), bool)
            keep[5, 1] = False
            assert np.isnan(rpn[5, 1]) and not np.isnan(rpn[keep]).any()
            np.testing.assert_array_equal(o[:, :, 0], samples[:, :, 0])
    P.close()


def test_pair_rejected_where_not_built():
    import torch
    from paper_2608_25666_amd import Projector, PrismError, options, Batch
    r = W.make_request(98, N=16, H=12, nj=2, dt=0.05, kind="white")   # H < 16
    P = Projector(r.H, r.nj, r.dt, r.bounds)
    x = torch.from_numpy(r.samples).cuda()
    with pytest.raises(PrismError) as e:
        P.solve(x, r.q0, r.v0, 10, opts=options(tile_waves=2))
    assert e.value.status == -6
    with pytest.raises(PrismError) as e:
        P.solve(x, r.q0, r.v0, 10, opts=options(tile_waves=3))
    assert e.value.status == -1
    r2 = W.make_request(99, N=16, H=50, nj=2, dt=0.05, kind="white")
    P2 = Projector(r2.H, r2.nj, r2.dt, r2.bounds)
    x2 = torch.from_numpy(r2.samples).cuda()
    q = torch.zeros((16, 2, 4, 50), dtype=torch.float32, device="cuda")
    with pytest.raises(PrismError):
        P2.solve(x2, r2.q0, r2.v0, 10, opts=options(tile_waves=2), state_out=q)
    B = Batch()
    with pytest.raises(PrismError):
        B.solve([dict(proj=P2, samples=x2, q0=r2.q0, v0=r2.v0, iters=10)],
                opts=options(tile_waves=2))
    P.close()
    P2.close()
