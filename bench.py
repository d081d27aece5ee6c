#!/usr/bin/env python3
"""Benchmark: projected trajectories per second at residual <= 1e-3 on one MI355X.

Workload (default): 2 arms x 6 joints = 12 joints, N = 2048 sampled velocity
trajectories, horizon H = 50, dt = 0.02 s, |q| <= 2 pi, |v| <= 3.14, |a| <= 8,
|j| <= 60; samples = smooth three-sinusoid base + N(0, 0.5^2) noise; rho = 1.
A step projects the whole batch until every 16-sample group of each joint has
max(r_primal, r_dual) <= 1e-3 (checked every 10 iterations, capped at 20000).
Inputs are resident in HBM before timing starts.

Prints one JSON line. Extra fields: per-step p50/p99 latency, iteration
statistics, the fixed-100-iteration throughput, a roofline object for the
solve kernel (timed live with HIP events on the solve's stream) and the FP64
oracle timed on the host cores on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|bf16|fp16]
                    [--alpha A] [--no-cpu-baseline] [--iters-cap C] [--workload mpc|long|uneven|serve|sigma|plan]

--workload long: 12 joints, N = 8192, H = 100 (same generator).
--workload serve: 32 controllers with the uneven requests' sizes issue Poisson requests at 20 Hz
each for --duration seconds into the continuous-batching server (warm start by
shift, HBM-budget admission); `value` is the served throughput and latency is
arrival to completion.
--workload sigma: the single-joint diagnostic of Sec. III-C: 200,000 white-noise
sequences (H = 15, dt = 0.1, sigma = --sigma, v0 = 0, |v| <= 1, |a| <= 2, |j| <= 4)
projected with one joint; reports the projected spread and the FP64 feasibility.
--workload plan: one optimizer iteration (prism_plan_step) per step on the default
batch shape: draw 2048 samples from N(nu, diag sigma^2) on the device, project them to
residual <= 1e-3, score them (tracking cost), softmax weights, mean/variance update.
--workload uneven: 64 requests with H in {20, 50, 100}, N in {128, 512, 2048, 4096},
6 or 12 joints and dt in {0.02, 0.05}, each with its own factor, projected in one
prism_proj_solve_batch call per step (FP32 and BF16 both timed; `value` is the
--precision one).
"""

from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_F32_TFLOPS = 157.3
PEAK_MFMA_B16_TFLOPS = 2500.0
# FP32 VALU issue: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane operations per second
# (one add/sub/max/med3/fma per lane per cycle; packed FP32 is not used).
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# FP64: dense matrix 78.6 TFLOP/s; vector FP64 issues at the same lane rate as FP32
# (78.6 TFLOP/s counting an FMA as two), so PEAK_VALU_TOPS lane operations per second.
PEAK_MFMA_F64_TFLOPS = 78.6


def valu_ops_per_col_iter(H: int) -> float:
    """Algorithmic FP32 VALU operations of one column-iteration.

    Forward rows C x: position prefix sums (H), acceleration (H) and jerk (H)
    differences. Row update on 4H-1 rows: t, z = clip(t), q, w (5 each).
    Transpose C^T w: position suffix sums (H), jerk/acceleration combination
    (2H) and difference (H), block sums (2H). Defect d: 3H.
    """
    return 3 * H + 5 * (4 * H - 1) + 6 * H + 3 * H


def mfma_flops_per_col_iter(H: int) -> float:
    """x += K d with the nonzero (H-1) x (H-1) block of K."""
    return 2.0 * (H - 1) ** 2


def literal_valu_ops_per_col_pass(H: int) -> float:
    """Algorithmic FP64 vector operations of one printed Bregman pass on one column.

    Rows s = C x at x: position prefix sums, acceleration and jerk differences (3H).
    Step 1 and the right-hand side of Step 2 in row form: m = min(ub, s) + max(lb, s)
    on 4H-1 rows (3 each); C^T W m: position suffix sums (H), one weighted
    accumulation per row into its step (4H), acceleration/jerk stencils (3H); rhs and
    t = w + delta/2 u (2H). Step 3: rows at x' (3H), C^T W s' (8H), w update (H).
    """
    return 3 * H + 3 * (4 * H - 1) + 8 * H + 2 * H + 3 * H + 8 * H + H


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="fp32", choices=["fp32", "bf16", "fp16"])
    ap.add_argument("--alpha", type=float, default=1.8)
    ap.add_argument("--weights", default="default", choices=["default", "unit"],
                    help="block penalty weights: prism_default_block_weights(H) or all ones")
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--iters-cap", type=int, default=20000)
    ap.add_argument("--fp32-tail", type=int, default=0)
    ap.add_argument("--N", type=int, default=2048)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fixed-iters", type=int, default=0,
                    help="time a fixed iteration count instead of the residual target")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the fixed-100-iteration section (for single-mode profiles)")
    ap.add_argument("--cpu-sample", type=int, default=1536, help="samples (all joints) for the oracle")
    ap.add_argument("--workload", default="mpc",
                    choices=["mpc", "long", "uneven", "serve", "sigma", "plan", "literal"])
    ap.add_argument("--passes", type=int, default=20, help="literal: printed Bregman passes")
    ap.add_argument("--delta", type=float, default=1.0, help="literal: penalty delta")
    ap.add_argument("--sigma", type=float, default=1.0, help="sigma: sampling sigma")
    ap.add_argument("--duration", type=float, default=60.0, help="serve: seconds of arrivals")
    ap.add_argument("--controllers", type=int, default=32, help="serve: controllers")
    ap.add_argument("--rate", type=float, default=20.0, help="serve: requests/s per controller")
    ap.add_argument("--max-inflight", type=int, default=4, help="serve: launches in flight")
    ap.add_argument("--max-batch", type=int, default=64, help="serve: requests per launch")
    ap.add_argument("--budget-gb", type=float, default=4.0, help="serve: warm-state pool")
    ap.add_argument("--grid-share", type=int, default=75, help="serve: percent of workgroup "
                    "slots one launch may take")
    ap.add_argument("--no-side", action="store_true", help="uneven/serve/sigma/plan: skip the "
                    "second precision")
    ap.add_argument("--cold", action="store_true", help="serve: no warm start (sample "
                    "counts alternate so no request matches its predecessor)")
    ap.add_argument("--copy-calibrate-mb", type=int, default=0,
                    help="first run a plain device copy of this many MiB (3 times): its "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the traffic figures")
    return ap.parse_args()


def kernel_source_sha(literal: bool = False) -> str:
    """sha256 over the device sources of a kernel, as recorded beside the rocprofv3
    counters in profiles/traffic.json: kernel_args.h with admm_*.h and admm_*.hip for
    the projection kernels, kernel_args.h with literal.hip for the printed iteration."""
    import hashlib
    d = os.path.join(ROOT, "paper_2608_25666_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if literal:
            own = f in ("kernel_args.h", "literal.hip")
        else:
            own = f == "kernel_args.h" or (f.startswith("admm_") and f[-2:] in (".h", "ip"))
        if own:
            h.update(f.encode())
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key: str, sha: str = None):
    """HBM bytes per launch from the committed FETCH_SIZE / WRITE_SIZE counters, or None
    when none were taken for this workload or the kernel sources changed since."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
            t = json.load(fh).get(key)
    except (OSError, ValueError):
        return None
    if not t or t.get("source_sha256") != (sha or kernel_source_sha()):
        return None
    return 1024.0 * (t["fetch_kib_per_dispatch"] * t["fetch_factor"] +
                     t["write_kib_per_dispatch"] * t["write_factor"])


def _oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return int(max([i.get("num_threads", 1) for i in threadpool_info()] + [1]))
    except Exception:
        return 1


def cpu_baseline(req, tol, check_every, cap, alpha, nsamp, weights):
    """The FP64 oracle on the first nsamp samples (all joints), timed on the host."""
    from oracle import admm
    S = req.samples[:nsamp]
    chunk = 32
    itmax = 0
    t0 = time.perf_counter()
    for c0 in range(0, S.shape[0], chunk):
        O = admm.solve_request(S[c0:c0 + chunk], req.H, req.dt, req.bounds, req.q0, req.v0,
                               rho=req.rho, alpha=alpha, iters=cap, tol=tol,
                               check_every=check_every, weights=weights)
        itmax = max(itmax, int(O.iters.max()))
    dt = time.perf_counter() - t0
    return {"value": S.shape[0] / dt, "unit": "trajectories/s", "cores": _oracle_threads(),
            "kind": "oracle",
            "sample": f"first {S.shape[0]} samples x {req.nj} joints of the benchmark batch "
                      f"(oracle called on {chunk} samples at a time), FP64 NumPy oracle to "
                      f"residual <= {tol:g} (check every {check_every}); {dt:.1f} s; max group "
                      f"iterations {itmax}"}


def cpu_baseline_batch(reqs, tol, check_every, cap, alpha, per_req, weights_of):
    """The FP64 oracle on the first per_req samples of every request, timed on the host."""
    from oracle import admm
    n = 0
    t0 = time.perf_counter()
    for r in reqs:
        S = r.samples[:per_req]
        admm.solve_request(S, r.H, r.dt, r.bounds, r.q0, r.v0, rho=r.rho, alpha=alpha, iters=cap,
                           tol=tol, check_every=check_every, weights=weights_of(r))
        n += S.shape[0]
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "trajectories/s", "cores": _oracle_threads(), "kind": "oracle",
            "sample": f"first {per_req} samples of each of the {len(reqs)} requests ({n} "
                      f"trajectories), FP64 NumPy oracle to residual <= {tol:g}; {dt:.1f} s"}


def roofline(col_iters_by_H, kern_s, prec_is_f32):
    """Roofline object for the solve kernel: algorithmic VALU and MFMA work of the
    column-iterations actually run, over the kernel's measured time."""
    valu = sum(valu_ops_per_col_iter(H) * c for H, c in col_iters_by_H.items())
    mflop = sum(mfma_flops_per_col_iter(H) * c for H, c in col_iters_by_H.items())
    peak_mfma = PEAK_MFMA_F32_TFLOPS if prec_is_f32 else PEAK_MFMA_B16_TFLOPS
    t_valu = valu / (PEAK_VALU_TOPS * 1e12)
    t_mfma = mflop / (peak_mfma * 1e12)
    if t_valu >= t_mfma:
        ach = valu / kern_s / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_VALU_TOPS}
    else:
        ach = mflop / kern_s / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": peak_mfma, "unit": "TFLOP/s",
                "frac": ach / peak_mfma}
    roof["traffic"] = None
    roof["mfma_util"] = mflop / kern_s / 1e12 / peak_mfma
    return roof


def _timed(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        fn()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall, np.array([s.elapsed_time(e) for s, e in ev])


def run_batch(a):
    """Uneven batch: 64 requests, one prism_proj_solve_batch call per step."""
    import torch
    import workloads as W
    from paper_2608_25666_amd import Batch, Projector, options, PREC_FP32, PREC_BF16, PREC_FP16
    reqs = W.uneven_requests()
    dev = torch.device("cuda:0")
    handles = {}
    for r in reqs:
        key = (r.H, r.nj, r.dt)
        if key not in handles:
            handles[key] = Projector(r.H, r.nj, r.dt, r.bounds, r.rho,
                                     weights=None if a.weights == "unit" else "default")
    xs = [torch.from_numpy(r.samples).to(dev) for r in reqs]
    outs = [torch.empty_like(x) for x in xs]
    rps = [torch.empty((r.N, r.nj), dtype=torch.float32, device=dev) for r in reqs]
    rds = [torch.empty_like(t) for t in rps]
    its = [torch.empty((r.N, r.nj), dtype=torch.int32, device=dev) for r in reqs]
    B = Batch()
    stream = torch.cuda.current_stream()
    fixed = a.fixed_iters > 0
    n_it = a.fixed_iters if fixed else a.iters_cap
    total_traj = sum(r.N for r in reqs)

    def measure(prec):
        opts = options(precision=prec, alpha=a.alpha, tol=0.0 if fixed else a.tol,
                       check_every=a.check_every, fp32_tail=a.fp32_tail)
        items = [dict(proj=handles[(r.H, r.nj, r.dt)], samples=x, q0=r.q0, v0=r.v0, iters=n_it,
                      out=o, r_primal=rp, r_dual=rd, iters_out=it)
                 for r, x, o, rp, rd, it in zip(reqs, xs, outs, rps, rds, its)]
        wall, per = _timed(lambda: B.solve(items, opts=opts, stream=stream), a.steps, a.warmup,
                           stream)
        col_iters = {}
        worst, conv, itmax, itsum, ncol = 0.0, 0, 0, 0.0, 0
        for r, rp, rd, it in zip(reqs, rps, rds, its):
            i = it.cpu().numpy()
            res = np.maximum(rp.cpu().numpy(), rd.cpu().numpy())
            col_iters[r.H] = col_iters.get(r.H, 0.0) + float(i.sum())
            conv += int((res <= a.tol).sum())
            ncol += res.size
            itmax = max(itmax, int(i.max()))
            itsum += float(i.sum())
        ms = wall * 1e3 / a.steps
        roof = roofline(col_iters, float(per.mean()) * 1e-3, prec == PREC_FP32)
        return {"value": total_traj / (ms * 1e-3), "ms_per_step": ms,
                "latency_ms": {"p50": float(np.percentile(per, 50)),
                               "p99": float(np.percentile(per, 99))},
                "iterations": {"max": itmax, "mean": itsum / ncol, "converged_frac": conv / ncol},
                "roofline": roof}

    main_prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]
    other = PREC_BF16 if main_prec == PREC_FP32 else PREC_FP32
    m = measure(main_prec)
    o = measure(other)
    shapes = sorted({(r.H, r.nj, r.dt) for r in reqs})
    line = {
        "metric": ("projected trajectories/sec at residual <=1e-3" if not fixed else
                   f"projected trajectories/sec at {a.fixed_iters} iterations"),
        "value": m["value"], "unit": "trajectories/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": m["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_prec == PREC_FP32 else ("bf16+f32" if main_prec == PREC_BF16
                                                         else "f16+f32"),
        "data": "synthetic",
        "config": {"workload": "uneven batch in one persistent launch: 64 requests, H in "
                               "{20,50,100}, N in {128,512,2048,4096}, 6 or 12 joints, dt in "
                               "{0.02,0.05}, own factor each, smooth 3-sinusoid + N(0,0.5^2) "
                               "samples, residual <= 1e-3",
                   "requests": len(reqs), "trajectories": total_traj,
                   "distinct_factors": len(shapes), "alpha": a.alpha, "precision": a.precision,
                   "tol": a.tol, "check_every": a.check_every, "iters_cap": a.iters_cap},
        "latency_ms": m["latency_ms"], "iterations": m["iterations"], "roofline": m["roofline"],
        "side_by_side": {("bf16" if other == PREC_BF16 else "fp32"): o},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_batch(
            reqs, a.tol, a.check_every, a.iters_cap, a.alpha, max(1, a.cpu_sample // 64),
            lambda r: handles[(r.H, r.nj, r.dt)].weights)
    print(json.dumps(line), flush=True)


def run_serve(a):
    """Serving: Poisson arrivals from many controllers into prism_server."""
    import torch
    from workloads import recipes as WC
    from paper_2608_25666_amd import Projector, Server, now_ns, options
    from paper_2608_25666_amd import PREC_FP32, PREC_BF16, PREC_FP16
    ctrls = WC.serving_controllers(n_controllers=a.controllers, rate_hz=a.rate,
                                   duration_s=a.duration)
    dev = torch.device("cuda:0")
    n_sets = 8
    handles = {}
    for c in ctrls:
        key = (c.H, c.nj, c.dt)
        if key not in handles:
            handles[key] = Projector(c.H, c.nj, c.dt, WC.UR5E_BIMANUAL_BOUNDS(c.nj), 1.0,
                                     weights=None if a.weights == "unit" else "default")
    # samples of steps 0..n_sets-1 per controller, resident before the run (request k uses
    # step k mod n_sets)
    sets = [[torch.from_numpy(WC.controller_samples(c, k)).to(dev) for k in range(n_sets)]
            for c in ctrls]
    if a.cold:       # every other request one sample short: never the predecessor's count
        sets = [[s if k % 2 == 0 else s[:-1] for k, s in enumerate(ss)] for ss in sets]
    arrivals = sorted((float(t), ci) for ci, c in enumerate(ctrls) for t in c.arrivals)
    n_req = len(arrivals)
    step_of = []
    cnt = [0] * len(ctrls)
    for _, ci in arrivals:
        step_of.append(cnt[ci])
        cnt[ci] += 1
    sizes = [sets[ci][(k + 1) % n_sets].shape[0] * ctrls[ci].nj
             for (_, ci), k in zip(arrivals, step_of)]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    it_all = torch.zeros(int(offs[-1]), dtype=torch.int32, device=dev)
    rp_all = torch.zeros(int(offs[-1]), dtype=torch.float32, device=dev)
    rd_all = torch.zeros_like(rp_all)
    outs = [[torch.empty_like(sets[ci][0]), torch.empty_like(sets[ci][0])] for ci in range(len(ctrls))]

    main_prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]

    def one_run(prec):
        opts = options(precision=prec, alpha=a.alpha, tol=a.tol, check_every=a.check_every,
                       fp32_tail=a.fp32_tail if prec == PREC_FP32 else max(a.fp32_tail, 10))
        S = Server(budget=int(a.budget_gb * (1 << 30)), opts=opts, max_inflight=a.max_inflight,
                   max_batch=a.max_batch, grid_share=a.grid_share)
        ids = [S.add_controller(handles[(c.H, c.nj, c.dt)], c.N) for c in ctrls]
        # warm-up (untimed): every controller's step 0, so kernels are loaded and each
        # controller holds a warm state when the arrival clock starts
        warm = [S.submit(ids[ci], sets[ci][0], c.q0, c.v0, a.iters_cap, outs[ci][1])
                for ci, c in enumerate(ctrls)]
        for t in warm:
            S.wait(t, 120000)
            S.release(t)
        torch.cuda.synchronize()
        tickets = []
        lags = np.zeros(len(arrivals))
        import gc
        gc.collect()
        gc.disable()          # a collection pass over the live tickets stalls the submitter
        t0 = now_ns() + 20_000_000
        late = 0
        next_report = 5.0
        for i, ((t, ci), k) in enumerate(zip(arrivals, step_of)):
            if t >= next_report:
                print(f"[serve {a.precision if prec == main_prec else 'other'}] {t:.0f} s of "
                      f"arrivals, {i} requests submitted", file=sys.stderr, flush=True)
                next_report += 5.0
            due = t0 + int(t * 1e9)
            while True:
                d = due - now_ns()
                if d <= 0:
                    break
                if d > 2_000_000:
                    time.sleep((d - 1_000_000) / 1e9)
            lags[i] = (now_ns() - due) / 1e6
            late = max(late, now_ns() - due)
            x = sets[ci][(k + 1) % n_sets]
            o = outs[ci][k % 2][:x.shape[0]]
            sl = slice(int(offs[i]), int(offs[i + 1]))
            c = ctrls[ci]
            tickets.append(S.submit(ids[ci], x, c.q0, c.v0, a.iters_cap, o,
                                    r_primal=rp_all[sl].view(x.shape[0], c.nj),
                                    r_dual=rd_all[sl].view(x.shape[0], c.nj),
                                    iters_out=it_all[sl].view(x.shape[0], c.nj)))
        infos = [S.wait(t, 120000) for t in tickets]
        gc.enable()
        torch.cuda.synchronize()
        stats = S.stats()
        for t in tickets:
            S.release(t)
        S.close()
        lat = np.array([(inf["t_done_ns"] - (t0 + int(t * 1e9))) / 1e6
                        for inf, (t, _) in zip(infos, arrivals)])
        t_end = max(inf["t_done_ns"] for inf in infos)
        span = (t_end - t0) / 1e9
        traj = sum(sets[ci][(k + 1) % n_sets].shape[0] for (_, ci), k in zip(arrivals, step_of))
        it_np = it_all.cpu().numpy()
        res = np.maximum(rp_all.cpu().numpy(), rd_all.cpu().numpy())
        col_iters = {}
        for i, ((_, ci), k) in enumerate(zip(arrivals, step_of)):
            H = ctrls[ci].H
            col_iters[H] = col_iters.get(H, 0.0) + float(it_np[offs[i]:offs[i + 1]].sum())
        warm = float(np.mean([inf["warm"] for inf in infos]))
        return {"value": traj / span, "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                                     "p99": float(np.percentile(lat, 99)),
                                                     "max": float(lat.max())},
                "requests": n_req, "trajectories": int(traj), "span_s": span,
                "warm_frac": warm, "max_submit_lag_ms": late / 1e6,
                "submit_lag_ms": {"p50": float(np.percentile(lags, 50)),
                                  "p99": float(np.percentile(lags, 99))},
                "iterations": {"mean": float(it_np.mean()), "max": int(it_np.max()),
                               "converged_frac": float(np.mean(res <= a.tol))},
                "mean_batch": float(np.mean([inf["batch_size"] for inf in infos])),
                "launches": stats["launches"], "evictions": stats["evictions"],
                "max_concurrent_launches": stats["max_concurrent_launches"],
                "gpu_busy_work": roofline(col_iters, span, prec == PREC_FP32)}

    main_prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]
    other = PREC_BF16 if main_prec == PREC_FP32 else PREC_FP32
    m = one_run(main_prec)
    o = None if a.no_side else one_run(other)
    line = {
        "metric": "projected trajectories/sec at residual <=1e-3; p50/p99 request latency",
        "value": m["value"], "unit": "trajectories/s", "n_gpus": 1, "steps": m["requests"],
        "warmup": 0, "ms_per_step": m["span_s"] * 1e3 / max(1, m["requests"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if main_prec == PREC_FP32 else ("bf16+f32" if main_prec == PREC_BF16
                                                         else "f16+f32"),
        "data": "synthetic",
        "config": {"workload": f"serving: {len(ctrls)} controllers (uneven-request sizes), Poisson "
                               f"{a.rate:g} Hz each for {a.duration:g} s, warm start by shift, "
                               f"HBM-budget admission, residual <= {a.tol:g}",
                   "controllers": len(ctrls), "rate_hz": a.rate, "duration_s": a.duration,
                   "budget_gb": a.budget_gb, "max_inflight": a.max_inflight,
                   "max_batch": a.max_batch, "grid_share": a.grid_share, "alpha": a.alpha,
                   "precision": a.precision,
                   "cold": a.cold},
        "latency_ms": m["latency_ms"], "serving": {k: v for k, v in m.items()
                                                   if k not in ("value", "latency_ms")},
        "side_by_side": {("bf16" if other == PREC_BF16 else "fp32"): o},
    }
    print(json.dumps(line), flush=True)


def run_sigma(a):
    """sigma_eff diagnostic: project 200k single-joint white-noise sequences."""
    import torch
    import workloads as W
    from paper_2608_25666_amd import Projector, options, PREC_FP32, PREC_BF16, PREC_FP16
    H, dt = 15, 0.1
    z, b = W.sigma_eff_workload(H=H)
    P = Projector(H, 1, dt, b, 1.0, weights=None if a.weights == "unit" else "default")
    dev = torch.device("cuda:0")
    x = torch.from_numpy((a.sigma * z).astype(np.float32)[:, :, None]).to(dev)
    N = x.shape[0]
    out = torch.empty_like(x)
    rp = torch.empty((N, 1), dtype=torch.float32, device=dev)
    rd = torch.empty_like(rp)
    it = torch.empty((N, 1), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()

    def measure(prec):
        o = options(precision=prec, alpha=a.alpha, tol=a.tol, check_every=a.check_every,
                    fp32_tail=0 if prec == PREC_FP32 else 10)
        wall, per = _timed(lambda: P.solve(x, [0.0], [0.0], a.iters_cap, opts=o, out=out,
                                           r_primal=rp, r_dual=rd, iters_out=it, stream=stream),
                           a.steps, a.warmup, stream)
        viol = P.feasibility(out, [0.0], [0.0]).cpu().numpy()
        i = it.cpu().numpy()
        res = np.maximum(rp.cpu().numpy(), rd.cpu().numpy())
        return {"value": N / (wall / a.steps), "ms_per_step": wall * 1e3 / a.steps,
                "latency_ms": {"p50": float(np.percentile(per, 50)),
                               "p99": float(np.percentile(per, 99))},
                "sigma_eff_qp": float(out.double().std().item()),
                "max_violation": float(viol.max()),
                "iterations": {"max": int(i.max()), "mean": float(i.mean()),
                               "converged_frac": float(np.mean(res <= a.tol))},
                "roofline": roofline({H: float(i.sum())}, float(per.mean()) * 1e-3,
                                     prec == PREC_FP32)}

    main_prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]
    m = measure(main_prec)
    other = PREC_BF16 if main_prec == PREC_FP32 else PREC_FP32
    o = measure(other)
    line = {"metric": "projected trajectories/sec at residual <=1e-3", "value": m["value"],
            "unit": "trajectories/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32" if main_prec == PREC_FP32 else "bf16+f32", "data": "synthetic",
            "config": {"workload": f"sigma_eff diagnostic: 200000 single-joint N(0,{a.sigma:g}^2) "
                                   "sequences, H=15, dt=0.1, v0=0, |v|<=1, |a|<=2, |j|<=4, "
                                   f"residual <= {a.tol:g}", "sigma": a.sigma},
            "latency_ms": m["latency_ms"], "sigma_eff_qp": m["sigma_eff_qp"],
            "max_violation": m["max_violation"], "iterations": m["iterations"],
            "roofline": m["roofline"],
            "side_by_side": {("bf16" if other == PREC_BF16 else "fp32"): o}}
    print(json.dumps(line), flush=True)


def run_plan(a):
    """Optimizer iterations around the projection on the default batch shape."""
    import torch
    import workloads as W
    from paper_2608_25666_amd import Projector, options, PREC_FP32, PREC_BF16, PREC_FP16
    req = W.mpc_batch(N=a.N)
    H, nj, N = req.H, req.nj, req.N
    P = Projector(H, nj, req.dt, req.bounds, req.rho,
                  weights=None if a.weights == "unit" else "default")
    dev = torch.device("cuda:0")
    rng = np.random.Generator(np.random.PCG64(1))
    base = req.samples.mean(axis=0)                         # the batch's smooth base
    nu = torch.from_numpy(base.astype(np.float32)).to(dev)
    sigma = torch.full((H, nj), 0.5, dtype=torch.float32, device=dev)
    ref = torch.from_numpy((req.q0[None, :] + req.dt * np.cumsum(base, axis=0)
                            + 0.05 * rng.standard_normal((H, nj))).astype(np.float32)).to(dev)
    it = torch.empty((N, nj), dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    ws = None
    step_id = [0]

    def measure(prec):
        nonlocal ws
        o = options(precision=prec, alpha=a.alpha, tol=a.tol, check_every=a.check_every,
                    fp32_tail=0 if prec == PREC_FP32 else 10)

        def one():
            nonlocal ws
            step_id[0] += 1
            g = P.plan_step(nu, sigma, N, 7, step_id[0], req.q0, req.v0, ref, w_pos=10.0,
                            w_vel=0.1, tau=1.0, eps=1e-3, iters=a.iters_cap, opts=o,
                            iters_out=it, workspace=ws, stream=stream)
            ws = g["workspace"]
        wall, per = _timed(one, a.steps, a.warmup, stream)
        i = it.cpu().numpy()
        return {"value": N / (wall / a.steps), "ms_per_step": wall * 1e3 / a.steps,
                "latency_ms": {"p50": float(np.percentile(per, 50)),
                               "p99": float(np.percentile(per, 99))},
                "iterations": {"max": int(i.max()), "mean": float(i.mean())}}

    main_prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]
    m = measure(main_prec)
    other = PREC_BF16 if main_prec == PREC_FP32 else PREC_FP32
    o2 = measure(other)
    line = {"metric": "projected trajectories/sec at residual <=1e-3", "value": m["value"],
            "unit": "trajectories/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
            "ms_per_step": m["ms_per_step"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32" if main_prec == PREC_FP32 else "bf16+f32", "data": "synthetic",
            "config": {"workload": f"optimizer iteration: {N} samples drawn on the device from "
                                   f"N(nu, 0.5^2), {nj} joints, H={H}, dt={req.dt}, projection "
                                   f"to residual <= {a.tol:g}, tracking cost, softmax "
                                   "weights (tau 1), mean/variance update"},
            "latency_ms": m["latency_ms"], "iterations": m["iterations"],
            "side_by_side": {("bf16" if other == PREC_BF16 else "fp32"): o2}}
    print(json.dumps(line), flush=True)


def run_literal(a):
    """The printed Bregman iteration (fast feasible-sample mode, not the projection) on
    the default batch shape: a fixed number of FP64 passes."""
    import ctypes as C
    import torch
    import workloads as W
    from paper_2608_25666_amd import Projector, _lib as L
    req = W.mpc_batch(N=a.N)
    H, nj, N = req.H, req.nj, req.N
    P = Projector(H, nj, req.dt, req.bounds, req.rho, weights="default")
    dev = torch.device("cuda:0")
    x = torch.from_numpy(req.samples).to(dev)
    out = torch.empty_like(x)
    viol = torch.empty((N, nj), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    # arguments marshalled once, so the timed loop is the launch alone
    q0a = L.dbl_array(np.asarray(req.q0, dtype=np.float64))
    v0a = L.dbl_array(np.asarray(req.v0, dtype=np.float64))
    la = L.LiteralArgs()
    la.v_samples, la.x_init, la.v_out, la.violation = x.data_ptr(), None, out.data_ptr(), viol.data_ptr()
    la.N, la.iters, la.delta = N, a.passes, a.delta
    la.q0 = C.cast(q0a, C.POINTER(C.c_double))
    la.v0 = C.cast(v0a, C.POINTER(C.c_double))
    fn, h, sp = L.lib().prism_proj_literal, P.handle, C.c_void_p(stream.cuda_stream)

    def step():
        st = fn(h, C.byref(la), sp)
        if st != 0:
            L.check(st, "prism_proj_literal")

    wall, per = _timed(step, a.steps, a.warmup, stream)
    kern_s = float(per.mean()) * 1e-3
    colp = float(N) * nj * a.passes
    mflop = 2.0 * (H - 1) ** 2 * colp
    valu = literal_valu_ops_per_col_pass(H) * colp
    t_m = mflop / (PEAK_MFMA_F64_TFLOPS * 1e12)
    t_v = valu / (PEAK_VALU_TOPS * 1e12)
    if t_m >= t_v:
        ach = mflop / kern_s / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": PEAK_MFMA_F64_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / PEAK_MFMA_F64_TFLOPS}
    else:
        ach = valu / kern_s / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_VALU_TOPS}
    roof["traffic"] = measured_traffic(f"literal_N{N}_H{H}_J{nj}_{a.passes}passes",
                                       sha=kernel_source_sha(literal=True))
    roof["algorithmic_bytes"] = 2 * N * H * nj * 4 + N * nj * 8
    roof["valu_frac"] = valu / kern_s / 1e12 / PEAK_VALU_TOPS
    roof["mfma_frac"] = mflop / kern_s / 1e12 / PEAK_MFMA_F64_TFLOPS
    v = viol.cpu().numpy()
    line = {"metric": f"trajectories/sec through {a.passes} printed Bregman passes "
                      "(fast feasible-sample mode, not the projection)",
            "value": N / (wall / a.steps), "unit": "trajectories/s", "n_gpus": 1,
            "steps": a.steps, "warmup": a.warmup, "ms_per_step": wall * 1e3 / a.steps,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": f"printed Bregman iteration: {N} samples x {nj} joints, "
                                   f"H={H}, dt={req.dt}, {a.passes} passes, delta={a.delta:g}, "
                                   "FP64"},
            "kernel_ms": float(per.mean()),
            "violation": {"max": float(v.max()), "frac_le_1e-3": float(np.mean(v <= 1e-3))},
            "roofline": roof}
    if not a.no_cpu_baseline:
        from oracle import admm, problem
        t0 = time.perf_counter()
        for j in range(nj):
            admm.literal_joint(req.samples[:, :, j].astype(np.float64), H, req.dt,
                               problem.joint_limits(req.bounds, j), float(req.q0[j]),
                               float(req.v0[j]), delta=a.delta, iters=a.passes)
        dt_cpu = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": N / dt_cpu, "unit": "trajectories/s",
                                "cores": _oracle_threads(), "kind": "oracle",
                                "sample": f"the whole batch ({N} samples x {nj} joints), "
                                          f"oracle literal_joint, {dt_cpu:.1f} s"}
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark measures one GPU: every (sample, joint) "
                          "column is an independent QP with no exchange step, so a batch "
                          "shards by samples or requests across GPUs without communication; "
                          "run with --gpus 1"}))
        sys.exit(2)
    import torch
    import workloads as W
    from paper_2608_25666_amd import Projector, options, PREC_FP32, PREC_BF16, PREC_FP16

    if a.copy_calibrate_mb > 0:
        nbytes = a.copy_calibrate_mb << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if a.workload == "uneven":
        return run_batch(a)
    if a.workload == "serve":
        return run_serve(a)
    if a.workload == "sigma":
        return run_sigma(a)
    if a.workload == "plan":
        return run_plan(a)
    if a.workload == "literal":
        return run_literal(a)
    prec = {"fp32": PREC_FP32, "bf16": PREC_BF16, "fp16": PREC_FP16}[a.precision]
    req = W.long_horizon_batch() if a.workload == "long" else W.mpc_batch(N=a.N)
    dev = torch.device("cuda:0")
    P = Projector(req.H, req.nj, req.dt, req.bounds, req.rho,
                  weights=None if a.weights == "unit" else "default")
    x = torch.from_numpy(req.samples).to(dev)
    out = torch.empty_like(x)
    rp = torch.empty((req.N, req.nj), dtype=torch.float32, device=dev)
    rd = torch.empty_like(rp)
    it = torch.empty((req.N, req.nj), dtype=torch.int32, device=dev)
    fixed = a.fixed_iters > 0
    opts = options(precision=prec, alpha=a.alpha, tol=0.0 if fixed else a.tol,
                   check_every=a.check_every, fp32_tail=a.fp32_tail)
    n_it = a.fixed_iters if fixed else a.iters_cap
    stream = torch.cuda.current_stream()

    def step():
        P.solve(x, req.q0, req.v0, n_it, opts=opts, out=out, r_primal=rp, r_dual=rd,
                iters_out=it, stream=stream)

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(a.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record(stream)
        step()
        e.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([s.elapsed_time(e) for s, e in ev])            # ms, solve launch on its stream
    ms_step = wall * 1e3 / a.steps
    iters = it.cpu().numpy()
    res = np.maximum(rp.cpu().numpy(), rd.cpu().numpy())
    converged = float(np.mean(res <= a.tol))

    # fixed-count throughput (100 iterations)
    fixed_ms = float("nan")
    if not a.no_extras:
        fopts = options(precision=prec, alpha=a.alpha, fp32_tail=a.fp32_tail)
        for _ in range(2):
            P.solve(x, req.q0, req.v0, 100, opts=fopts, out=out, r_primal=rp, r_dual=rd,
                    stream=stream)
        torch.cuda.synchronize()
        fe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(10)]
        for s, e in fe:
            s.record(stream)
            P.solve(x, req.q0, req.v0, 100, opts=fopts, out=out, r_primal=rp, r_dual=rd,
                    stream=stream)
            e.record(stream)
        torch.cuda.synchronize()
        fixed_ms = float(np.mean([s.elapsed_time(e) for s, e in fe]))

    # roofline of the solve kernel over the timed region
    H = req.H
    col_iters = float(iters.sum())
    valu = valu_ops_per_col_iter(H) * col_iters
    mflop = mfma_flops_per_col_iter(H) * col_iters
    kern_s = float(per.mean()) * 1e-3
    t_valu = valu / (PEAK_VALU_TOPS * 1e12)
    peak_mfma = PEAK_MFMA_F32_TFLOPS if prec == PREC_FP32 else PEAK_MFMA_B16_TFLOPS
    t_mfma = mflop / (peak_mfma * 1e12)
    if t_valu >= t_mfma:
        ach = valu / kern_s / 1e12
        roof = {"bound": "alu", "achieved": ach, "peak": PEAK_VALU_TOPS, "unit": "TFLOP/s",
                "frac": ach / PEAK_VALU_TOPS}
    else:
        ach = mflop / kern_s / 1e12
        roof = {"bound": "mfma", "achieved": ach, "peak": peak_mfma, "unit": "TFLOP/s",
                "frac": ach / peak_mfma}
    roof["traffic"] = None
    if a.workload == "mpc" and req.N == 2048 and prec == PREC_FP32 and not fixed:
        roof["traffic"] = measured_traffic("mpc_N2048_H50_J12_fp32_residual")
    roof["algorithmic_bytes"] = req.N * req.nj * H * 8 + req.N * req.nj * 12
    roof["mfma_util"] = mflop / kern_s / 1e12 / peak_mfma
    roof["hbm_gbs"] = roof["algorithmic_bytes"] / kern_s / 1e9
    fixed_cols = req.N * req.nj * 100
    fixed_valu = valu_ops_per_col_iter(H) * fixed_cols / (fixed_ms * 1e-3) / 1e12
    fixed_mfma = mfma_flops_per_col_iter(H) * fixed_cols / (fixed_ms * 1e-3) / 1e12

    line = {
        "metric": ("projected trajectories/sec at residual <=1e-3" if not fixed else
                   f"projected trajectories/sec at {a.fixed_iters} iterations"),
        "value": req.N / (ms_step * 1e-3),
        "unit": "trajectories/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == PREC_FP32 else ("bf16+f32" if prec == PREC_BF16 else "f16+f32"),
        "data": "synthetic",
        "config": {"workload": f"projection QP, 12 joints, N={req.N}, H={H}, dt={req.dt}, rho=1, "
                               "smooth 3-sinusoid + N(0,0.5^2) samples, residual <= 1e-3",
                   "N": req.N, "H": H, "joints": req.nj, "dt": req.dt, "rho": req.rho,
                   "alpha": a.alpha, "block_weights": P.weights or (1.0, 1.0, 1.0, 1.0),
                   "precision": a.precision, "tol": a.tol,
                   "check_every": a.check_every, "iters_cap": a.iters_cap},
        "latency_ms": {"p50": float(np.percentile(per, 50)), "p99": float(np.percentile(per, 99))},
        "iterations": {"max": int(iters.max()), "mean": float(iters.mean()),
                       "p50": float(np.median(iters)), "converged_frac": converged},
        "fixed_100_iters": {"ms": fixed_ms, "trajectories_per_s": req.N / (fixed_ms * 1e-3),
                            "valu_tops": fixed_valu, "valu_frac": fixed_valu / PEAK_VALU_TOPS,
                            "mfma_tflops": fixed_mfma, "mfma_frac": fixed_mfma / peak_mfma},
        "roofline": roof,
    }
    if a.no_extras:
        line["fixed_100_iters"] = None
    elif prec == PREC_FP32 and not fixed:
        # the reduced-precision forms on the same batch at the same residual target
        side = {}
        for name, p2 in (("bf16", PREC_BF16), ("fp16", PREC_FP16)):
            o2 = options(precision=p2, alpha=a.alpha, tol=a.tol, check_every=a.check_every,
                         fp32_tail=10)
            w2, per2 = _timed(lambda: P.solve(x, req.q0, req.v0, n_it, opts=o2, out=out,
                                              r_primal=rp, r_dual=rd, iters_out=it,
                                              stream=stream), a.steps, a.warmup, stream)
            res2 = np.maximum(rp.cpu().numpy(), rd.cpu().numpy())
            it2 = it.cpu().numpy()
            side[name + "+10fp32"] = {
                "value": req.N / (w2 / a.steps), "ms_per_step": w2 * 1e3 / a.steps,
                "latency_ms": {"p50": float(np.percentile(per2, 50)),
                               "p99": float(np.percentile(per2, 99))},
                "iterations": {"max": int(it2.max()), "mean": float(it2.mean()),
                               "converged_frac": float(np.mean(res2 <= a.tol))}}
        line["side_by_side"] = side
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(req, a.tol, a.check_every, a.iters_cap, a.alpha,
                                            a.cpu_sample, P.weights)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
