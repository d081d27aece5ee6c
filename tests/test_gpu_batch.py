"""Uneven batch in one persistent launch (prism_proj_solve_batch).

Each request keeps its own horizon, joint count, dt, bounds and factor. The
batched result of a request must equal what its own prism_proj_solve_ex call
gives (same tile code, same arithmetic order), and match the FP64 oracle at
the FP32 bar (1e-4 rad/s max-abs) on sampled requests.
"""

import numpy as np
import pytest

from oracle import admm
import workloads as W

pytestmark = pytest.mark.gpu


def _small_mix(seed, h_choices=(20, 50, 100), n_choices=(16, 37, 64), n_requests=10):
    return W.uneven_requests(seed=seed, n_requests=n_requests, n_choices=n_choices,
                              h_choices=h_choices, iters=100)


def _batch_and_single(reqs, iters, opts, weights="default", with_iters=False):
    import torch
    from paper_2608_25666_amd import Batch, Projector
    projs = [Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights=weights) for r in reqs]
    xs = [torch.from_numpy(np.ascontiguousarray(r.samples)).cuda() for r in reqs]
    its = [torch.zeros((r.N, r.nj), dtype=torch.int32, device="cuda") for r in reqs]
    B = Batch()
    outs = B.solve([dict(proj=P, samples=x, q0=r.q0, v0=r.v0, iters=iters,
                         iters_out=it if with_iters else None)
                    for P, x, r, it in zip(projs, xs, reqs, its)], opts=opts)
    torch.cuda.synchronize()
    batched = [(o.cpu().numpy(), rp.cpu().numpy(), rd.cpu().numpy(), it.cpu().numpy())
               for (o, rp, rd), it in zip(outs, its)]
    single = []
    for P, x, r in zip(projs, xs, reqs):
        it = torch.zeros((r.N, r.nj), dtype=torch.int32, device="cuda")
        o, rp, rd = P.solve(x, r.q0, r.v0, iters, opts=opts, iters_out=it if with_iters else None)
        torch.cuda.synchronize()
        single.append((o.cpu().numpy(), rp.cpu().numpy(), rd.cpu().numpy(), it.cpu().numpy()))
    ws = [P.weights for P in projs]
    B.close()
    for P in projs:
        P.close()
    return batched, single, ws


def _assert_same(batched, single, exact=True):
    for b, s in zip(batched, single):
        for u, v in zip(b, s):
            if exact:
                np.testing.assert_array_equal(u, v)
            else:
                np.testing.assert_allclose(u, v, atol=2e-6, rtol=0)


def test_batch_mpc_set_equals_single_solves_and_oracle():
    """Horizons 20/50/100 (one launch), sample counts with ragged tails, 6 or 12 joints."""
    from paper_2608_25666_amd import options
    reqs = _small_mix(3)
    assert len({r.H for r in reqs}) >= 2
    batched, single, ws = _batch_and_single(reqs, 100, options(alpha=1.6))
    _assert_same(batched, single)
    worst = 0.0
    for r, b, w in list(zip(reqs, batched, ws))[:4]:
        pick = np.unique(np.r_[0, 1, r.N - 1])
        O = admm.solve_request(r.samples[pick], r.H, r.dt, r.bounds, r.q0, r.v0, iters=100,
                               alpha=1.6, weights=w)
        err = np.abs(b[0][pick] - O.x).max()
        worst = max(worst, err)
        np.testing.assert_allclose(b[1][pick], O.r_p, atol=1e-4, rtol=1e-3)
        np.testing.assert_allclose(b[2][pick], O.r_d, atol=1e-4, rtol=1e-3)
    print(f"batch vs oracle worst max-abs {worst:.3e}")
    assert worst <= 1e-4


def test_batch_mixed_chunk_classes():
    """Horizons outside {20,50,100}: one launch per chunk class, still per-request exact."""
    from paper_2608_25666_amd import options
    reqs = _small_mix(4, h_choices=(2, 7, 33, 64, 128), n_choices=(5, 16, 40), n_requests=9)
    batched, single, ws = _batch_and_single(reqs, 60, options(alpha=1.6))
    _assert_same(batched, single)
    r, b, w = reqs[0], batched[0], ws[0]
    O = admm.solve_request(r.samples[:3], r.H, r.dt, r.bounds, r.q0, r.v0, iters=60,
                           alpha=1.6, weights=w)
    assert np.abs(b[0][:3] - O.x).max() <= 1e-4


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_batch_long_chunk_classes(prec):
    """Horizons 99..128 (chunks 25, 28, 30, 31, 32) take the four one-wave classes
    {25..28}, {29, 30}, {31}, {32}: per-request exact against the single solves, and
    one request of each chunk against the oracle (FP32 bar; reduced forms at their
    fixed-count bar)."""
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP32
    from test_gpu_forms import TOL_BF16_TAIL
    p = PREC_FP32 if prec == "fp32" else PREC_BF16
    reqs = _small_mix(5, h_choices=(99, 110, 117, 121, 128), n_choices=(5, 16, 40), n_requests=8)
    chunks = [(r.H + 3) // 4 for r in reqs]
    assert sorted(set(chunks)) == [25, 28, 30, 31, 32]
    o = options(alpha=1.6, precision=p, fp32_tail=0 if prec == "fp32" else 10)
    batched, single, ws = _batch_and_single(reqs, 60, o)
    _assert_same(batched, single)
    for c in sorted(set(chunks)):
        k = chunks.index(c)
        r, b, w = reqs[k], batched[k], ws[k]
        O = admm.solve_request(r.samples[:3], r.H, r.dt, r.bounds, r.q0, r.v0, iters=60,
                               alpha=1.6, weights=w)
        err = np.abs(b[0][:3] - O.x).max()
        print(f"chunk {c} (H={r.H}) {prec}: max-abs {err:.3e}")
        assert err <= (1e-4 if prec == "fp32" else TOL_BF16_TAIL)


@pytest.mark.parametrize("tol", [0.0, 1e-3])
@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_eight_wave_single_solves_equal_batch(prec, tol):
    """Single solves of the reduced forms at chunks 22..25 (H = 86, 90, 93, 97; ragged
    rows) run eight waves per workgroup; the batch runs the same tile code four waves per
    workgroup. Per request bit-identical, fixed count and residual mode; one request
    against the oracle at the fixed count."""
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP16
    from test_gpu_forms import TOL_BF16_TAIL
    from test_gpu_pair import TOL_F16_FIXED   # FP16 at a fixed count, alpha 1.8
    p = PREC_BF16 if prec == "bf16" else PREC_FP16
    reqs = _small_mix(11, h_choices=(86, 90, 93, 97), n_choices=(16, 37, 300), n_requests=8)
    assert sorted({(r.H + 3) // 4 for r in reqs}) == [22, 23, 24, 25]
    o = options(precision=p, fp32_tail=10, alpha=1.8, tol=tol)
    batched, single, ws = _batch_and_single(reqs, 2000 if tol > 0 else 100, o, with_iters=True)
    _assert_same(batched, single)
    if tol == 0.0:
        r, b, w = reqs[0], batched[0], ws[0]
        O = admm.solve_request(r.samples[:4], r.H, r.dt, r.bounds, r.q0, r.v0, iters=100,
                               alpha=1.8, weights=w)
        err = np.abs(b[0][:4] - O.x).max()
        print(f"H={r.H} {prec}: max-abs {err:.3e}")
        assert err <= (TOL_BF16_TAIL if prec == "bf16" else TOL_F16_FIXED)
    else:
        for b in batched:
            assert np.all(np.maximum(b[1], b[2]) <= 1e-3)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_batch_reduced_precision_equals_single(prec):
    from paper_2608_25666_amd import options, PREC_BF16, PREC_FP16
    p = PREC_BF16 if prec == "bf16" else PREC_FP16
    reqs = _small_mix(5, n_requests=6)
    batched, single, _ = _batch_and_single(reqs, 100, options(precision=p, fp32_tail=10, alpha=1.6))
    _assert_same(batched, single)


def test_batch_residual_mode_iteration_counts():
    """Residual-driven stopping per group of 16 samples inside the batch."""
    from paper_2608_25666_amd import options
    reqs = _small_mix(6, n_requests=6)
    batched, single, _ = _batch_and_single(reqs, 3000, options(alpha=1.6, tol=1e-3), with_iters=True)
    _assert_same(batched, single)
    for b in batched:
        assert np.all(np.maximum(b[1], b[2]) <= 1e-3)


def test_batch_empty_and_invalid_requests():
    import torch
    from paper_2608_25666_amd import Batch, PrismError, Projector
    r = W.make_request(7, N=20, H=20, nj=2, dt=0.05, kind="white")
    P = Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights="default")
    x = torch.from_numpy(np.ascontiguousarray(r.samples)).cuda()
    B = Batch()
    assert B.solve([]) == []
    empty = torch.zeros((0, r.H, r.nj), dtype=torch.float32, device="cuda")
    out = torch.full_like(x, 7.0)
    B.solve([dict(proj=P, samples=empty, q0=r.q0, v0=r.v0, iters=50),
             dict(proj=P, samples=x, q0=r.q0, v0=r.v0, iters=50, out=out)])
    torch.cuda.synchronize()
    ref, _, _ = P.solve(x, r.q0, r.v0, 50)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(out.cpu().numpy(), ref.cpu().numpy())
    # a request whose boundary state is infeasible rejects the whole call, nothing written
    out2 = torch.full_like(x, 7.0)
    bad_v0 = np.full(r.nj, 100.0)
    with pytest.raises(PrismError):
        B.solve([dict(proj=P, samples=x, q0=r.q0, v0=r.v0, iters=50, out=out2),
                 dict(proj=P, samples=x, q0=r.q0, v0=bad_v0, iters=50)])
    torch.cuda.synchronize()
    assert np.all(out2.cpu().numpy() == 7.0)
    B.close()
    P.close()


def test_batch_warm_shift_equals_single():
    """Batched requests that warm-start from a previous result advanced by one step."""
    import torch
    from paper_2608_25666_amd import Batch, Projector, options
    reqs = _small_mix(8, n_requests=5)
    o = options(alpha=1.6)
    projs = [Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights="default") for r in reqs]
    xs = [torch.from_numpy(np.ascontiguousarray(r.samples)).cuda() for r in reqs]
    prev, states = [], []
    for P, x, r in zip(projs, xs, reqs):
        q = torch.zeros((r.N, r.nj, 4, r.H), dtype=torch.float32, device="cuda")
        out, _, _ = P.solve(x, r.q0, r.v0, 30, opts=o, state_out=q)
        prev.append(out)
        states.append(q)
    flipped = [torch.flip(x, dims=[0]).contiguous() for x in xs]   # next step's samples
    B = Batch()
    outs = B.solve([dict(proj=P, samples=f, q0=r.q0, v0=r.v0, iters=40, x_warm=p, state_warm=q,
                         warm_shift=True)
                    for P, f, r, p, q in zip(projs, flipped, reqs, prev, states)], opts=o)
    singles = [P.solve(f, r.q0, r.v0, 40, opts=o, x_warm=p, state_warm=q, warm_shift=True)
               for P, f, r, p, q in zip(projs, flipped, reqs, prev, states)]
    torch.cuda.synchronize()
    for (bo, brp, brd), (so, srp, srd) in zip(outs, singles):
        np.testing.assert_array_equal(bo.cpu().numpy(), so.cpu().numpy())
        np.testing.assert_array_equal(brp.cpu().numpy(), srp.cpu().numpy())
    B.close()
    for P in projs:
        P.close()


def test_split_batch_orders_the_callers_stream():
    """A {20, 50, 100} batch runs its H = 20/50 launch on a stream forked from the
    caller's: work queued on the caller's stream after the call (here a copy of every
    output, with no device-wide synchronisation in between) must see the finished
    results of both launches, on a non-default stream and on two calls in a row."""
    import torch
    from paper_2608_25666_amd import Batch, Projector, options, PREC_FP32
    reqs = _small_mix(31, n_choices=(512, 1024), n_requests=6)
    assert {r.H for r in reqs} >= {100} and {r.H for r in reqs} & {20, 50}
    projs = [Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights="default") for r in reqs]
    xs = [torch.from_numpy(np.ascontiguousarray(r.samples)).cuda() for r in reqs]
    opts = options(precision=PREC_FP32, alpha=1.8, tol=1e-3, check_every=10)
    ref = []
    for P, x, r in zip(projs, xs, reqs):
        o, _, _ = P.solve(x, r.q0, r.v0, 5000, opts=opts)
        torch.cuda.synchronize()
        ref.append(o.cpu().numpy())
    B = Batch()
    s = torch.cuda.Stream()
    for rep in range(2):
        with torch.cuda.stream(s):
            outs = [torch.full_like(x, float("nan")) for x in xs]
            B.solve([dict(proj=P, samples=x, q0=r.q0, v0=r.v0, iters=5000, out=o)
                     for P, x, r, o in zip(projs, xs, reqs, outs)], opts=opts, stream=s)
            copies = [o.clone() for o in outs]      # queued on s behind the batch
        s.synchronize()
        for c, want in zip(copies, ref):
            np.testing.assert_array_equal(c.cpu().numpy(), want)
    B.close()
    for P in projs:
        P.close()


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_uneven_batch_bench_settings_sampled(prec):
    """The 64-request uneven batch in one call as the benchmark runs it: each request's
    default block weights (scaled by its jerk bound and dt), alpha 1.8, residual <= 1e-3
    checked every 10, reduced forms with 10 FP32 iterations after convergence. Every
    column must meet the tolerance; the first and last tiles of an H = 100 and an H = 50
    request at dt = 0.05 and of H = 100 and H = 20 requests at dt = 0.02, on their slowest
    joint and one other, against the oracle run to the reported counts (tests/stops.py)."""
    import torch
    from paper_2608_25666_amd import Batch, Projector, options, PREC_BF16, PREC_FP16, PREC_FP32
    from stops import check_residual_mode
    from test_gpu_forms import TOL_REDUCED_RESIDUAL
    p = {"fp32": PREC_FP32, "fp16": PREC_FP16, "bf16": PREC_BF16}[prec]
    reqs = W.uneven_requests()
    handles = {}
    items, outs = [], []
    for r in reqs:
        key = (r.H, r.nj, r.dt)
        if key not in handles:
            handles[key] = Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights="default")
        x = torch.from_numpy(r.samples).cuda()
        it = torch.zeros((r.N, r.nj), dtype=torch.int32, device="cuda")
        items.append(dict(proj=handles[key], samples=x, q0=r.q0, v0=r.v0, iters=20000, iters_out=it))
        outs.append(it)
    o = options(precision=p, alpha=1.8, tol=1e-3, check_every=10,
                fp32_tail=0 if prec == "fp32" else 10)
    B = Batch()
    res = B.solve(items, opts=o)
    torch.cuda.synchronize()
    for (x, rp, rd) in res:
        assert np.all(np.maximum(rp.cpu().numpy(), rd.cpu().numpy()) <= 1e-3)
    picks = {}
    for k, r in enumerate(reqs):
        key = (r.H, r.dt)
        if key in ((100, 0.05), (50, 0.05), (100, 0.02), (20, 0.02)) and key not in picks \
                and r.N >= 512:
            picks[key] = k
    assert len(picks) == 4
    for key, k in sorted(picks.items()):
        r = reqs[k]
        x, rp, rd = res[k]
        itg = outs[k].cpu().numpy()
        rows = np.r_[np.arange(0, 16), np.arange(r.N - 16, r.N)]
        joints = sorted({int(np.argmax(itg.max(axis=0))), 0})
        w = handles[(r.H, r.nj, r.dt)].weights
        check_residual_mode(x.cpu().numpy()[rows], rp.cpu().numpy()[rows], rd.cpu().numpy()[rows],
                            itg[rows], rows, r.samples, r.H, r.dt, r.bounds, r.q0, r.v0,
                            tol=1e-3, check_every=10, cap=20000, alpha=1.8, weights=w,
                            xbar=1e-4 if prec == "fp32" else TOL_REDUCED_RESIDUAL,
                            check_stops=prec == "fp32",
                            label=f"uneven request {k} H={r.H} dt={r.dt} {prec}", joints=joints)
    B.close()
    for P in handles.values():
        P.close()


def test_reduced_form_divergence_restarts_in_fp32():
    """Near alpha = 2 the BF16 x-update's rounding can outweigh the contraction: at 1.95
    the iterates of some tiles of the uneven batch diverge (measured with no guard: NaN
    on 5816 columns, also at a fixed 3000 iterations; at 1.9 on 17; FP32 and FP16 none).
    In residual mode a tile whose residual rises 64x above its lowest restarts from the
    sample with a cold state in the FP32 form, and one whose residual sets no new low
    for 500 iterations goes on in FP32 (with the restart rule alone, 213,832 columns
    still stalled above tol until the cap). So every column is finite and meets the
    tolerance; a restarted tile's result is bit for bit the FP32 form's, after a whole
    number of check periods more iterations (the ones it abandoned); the slowest tile's
    columns agree with the oracle run to the reported counts; and the same request alone
    through the one-wave and the two-wave tile kernels does the same."""
    import torch
    from paper_2608_25666_amd import Batch, Projector, options, PREC_BF16, PREC_FP32
    from stops import check_residual_mode
    from test_gpu_forms import TOL_REDUCED_RESIDUAL
    alpha, cap, ce = 1.95, 20000, 10
    reqs = W.uneven_requests()
    handles = {}
    for r in reqs:
        key = (r.H, r.nj, r.dt)
        if key not in handles:
            handles[key] = Projector(r.H, r.nj, r.dt, r.bounds, r.rho, weights="default")
    xs = [torch.from_numpy(r.samples).cuda() for r in reqs]
    B = Batch()

    def run(prec):
        its = [torch.zeros((r.N, r.nj), dtype=torch.int32, device="cuda") for r in reqs]
        res = B.solve([dict(proj=handles[(r.H, r.nj, r.dt)], samples=x, q0=r.q0, v0=r.v0,
                            iters=cap, iters_out=it) for r, x, it in zip(reqs, xs, its)],
                      opts=options(precision=prec, alpha=alpha, tol=1e-3, check_every=ce,
                                   fp32_tail=0 if prec == PREC_FP32 else 10))
        torch.cuda.synchronize()
        return [(x.cpu().numpy(), np.maximum(rp.cpu().numpy(), rd.cpu().numpy()), it.cpu().numpy())
                for (x, rp, rd), it in zip(res, its)]

    ref, red = run(PREC_FP32), run(PREC_BF16)
    restarted, top = 0, (0, 0)
    for k, (r, (xf, _, itf), (xb, res, itb)) in enumerate(zip(reqs, ref, red)):
        assert not np.isnan(xb).any()
        assert np.all(res <= 1e-3)
        if itb.max() > top[0]:
            top = (int(itb.max()), k)
        for t0 in range(0, r.N, 16):
            for j in range(r.nj):
                cols = slice(t0, min(t0 + 16, r.N))
                d = itb[cols, j] - itf[cols, j]
                if np.array_equal(xb[cols, :, j], xf[cols, :, j]) and d[0] > 0:
                    assert np.all(d == d[0]) and d[0] % ce == 0
                    restarted += 1
    print(f"alpha {alpha} bf16: tiles restarted in FP32 {restarted}, max iterations {top[0]} "
          f"(request {top[1]})")
    assert restarted > 0
    assert top[0] < cap // 2     # measured 5620 (the cap was reached without the guards)
    # the slowest tile against the oracle: a restarted one as the FP32 form it became
    # (the oracle run to the FP32 counts, FP32 bar and stop points), else at the
    # reduced form's residual-mode bar
    k = top[1]
    r = reqs[k]
    xb, res, itg = red[k]
    xf, _, itf = ref[k]
    col, jnt = np.unravel_index(int(np.argmax(itg)), itg.shape)
    rows = np.arange((col // 16) * 16, min((col // 16) * 16 + 16, r.N))
    P = handles[(r.H, r.nj, r.dt)]
    was_restarted = np.array_equal(xb[rows, :, jnt], xf[rows, :, jnt])
    check_residual_mode(xb[rows], res[rows], res[rows], (itf if was_restarted else itg)[rows],
                        rows, r.samples, r.H, r.dt, r.bounds, r.q0, r.v0, tol=1e-3,
                        check_every=ce, cap=cap, alpha=alpha, weights=P.weights,
                        xbar=1e-4 if was_restarted else TOL_REDUCED_RESIDUAL,
                        check_stops=was_restarted,
                        label=f"slowest tile of request {k} (H={r.H}, restarted {was_restarted})",
                        joints=[int(jnt)])
    for tw in (1, 2):
        it = torch.zeros((r.N, r.nj), dtype=torch.int32, device="cuda")
        x1, rp1, rd1 = P.solve(xs[k], r.q0, r.v0, cap, iters_out=it,
                               opts=options(precision=PREC_BF16, alpha=alpha, tol=1e-3,
                                            check_every=ce, fp32_tail=10, tile_waves=tw))
        torch.cuda.synchronize()
        x1 = x1.cpu().numpy()
        assert not np.isnan(x1).any()
        assert np.all(np.maximum(rp1.cpu().numpy(), rd1.cpu().numpy()) <= 1e-3)
        print(f"request {k} alone, tile_waves {tw}: max iterations {int(it.max().item())}")
        assert int(it.max().item()) < cap // 2
        if tw == 1:
            np.testing.assert_array_equal(x1, xb)
            np.testing.assert_array_equal(it.cpu().numpy(), itg)
    B.close()
    for P in handles.values():
        P.close()
