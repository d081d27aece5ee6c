"""prism_plan_step_static, the optimizer step that allocates nothing (its workspace and
tile-queue counters live in the library's static device scratch), against
prism_plan_step with a caller workspace: the same kernels on the same inputs, so every
output must be bit-identical, on two calls in a row with the second one smaller (the
scratch keeps the first call's contents). A request beyond the scratch capacity is
refused with PRISM_ETOOLARGE and writes nothing. Through the C ABI (ctypes)."""

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _outputs(N, H, nj, dev, fill):
    import torch
    f32 = torch.float32
    return {"x": torch.full((N, H, nj), fill, dtype=f32, device=dev),
            "cost": torch.full((N,), fill, dtype=torch.float64, device=dev),
            "omega": torch.full((N,), fill, dtype=torch.float64, device=dev),
            "nu": torch.full((H, nj), fill, dtype=f32, device=dev),
            "var": torch.full((H, nj), fill, dtype=f32, device=dev),
            "best": torch.full((1,), -7, dtype=torch.int32, device=dev),
            "samples": torch.full((N, H, nj), fill, dtype=f32, device=dev),
            "iters": torch.full((N, nj), -7, dtype=torch.int32, device=dev),
            "rp": torch.full((N, nj), fill, dtype=f32, device=dev),
            "rd": torch.full((N, nj), fill, dtype=f32, device=dev)}


def _call(P, ws, outs, N, seed, stream_id, r, nu_t, sigma_t, ref_t, opts, static):
    return P.plan_step(nu_t, sigma_t, N, seed, stream_id, r.q0, r.v0, ref_t, w_pos=10.0,
                       w_vel=0.1, tau=1.0, eps=1e-3, iters=20000, opts=opts,
                       samples_out=outs["samples"], r_primal=outs["rp"], r_dual=outs["rd"],
                       iters_out=outs["iters"], static=static, outputs=outs, workspace=ws)


def test_static_plan_step_matches_workspace_version():
    import torch
    from paper_2608_25666_amd import Projector, options, PREC_BF16, PREC_FP32
    H, nj, dt = 50, 12, 0.02
    r = W.make_request(81, N=1, H=H, nj=nj, dt=dt, kind="smooth")
    P = Projector(H, nj, dt, r.bounds, 1.0, weights="default")
    dev = torch.device("cuda")
    rng = np.random.default_rng(81)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    nu_t = t(0.3 * rng.normal(size=(H, nj)))
    sigma_t = t(np.full((H, nj), 0.5))
    ref_t = t(r.q0[None, :] + np.cumsum(np.full((H, nj), 0.02), axis=0))
    calls = [(1536, PREC_FP32, 5), (200, PREC_BF16, 6)]     # the second call is smaller
    for k, (N, prec, seed) in enumerate(calls):
        o = options(precision=prec, alpha=1.8, tol=1e-3, check_every=10,
                    fp32_tail=0 if prec == PREC_FP32 else 10)
        a = _outputs(N, H, nj, dev, 0.0)
        b = _outputs(N, H, nj, dev, 123.0)
        _call(P, None, a, N, seed, k, r, nu_t, sigma_t, ref_t, o, static=False)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        free_before = torch.cuda.mem_get_info()[0]
        _call(P, None, b, N, seed, k, r, nu_t, sigma_t, ref_t, o, static=True)
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        if k > 0:
            assert torch.cuda.mem_get_info()[0] == free_before
        for name in a:
            np.testing.assert_array_equal(a[name].cpu().numpy(), b[name].cpu().numpy(),
                                          err_msg=f"call {k}: {name}")
        assert np.all(np.maximum(b["rp"].cpu().numpy(), b["rd"].cpu().numpy()) <= 1e-3)
        print(f"call {k}: N={N}, iterations {int(b['iters'].max())}, outputs bit-identical")
    P.close()


def test_static_plan_step_refuses_too_large_requests():
    import torch
    from paper_2608_25666_amd import Projector, PrismError, options
    from paper_2608_25666_amd import _lib as L
    H, nj, dt = 50, 12, 0.02
    N = 92667                       # the first N whose workspace exceeds the scratch
    assert L.lib().prism_plan_workspace_bytes(H, nj, N) > L.PLAN_STATIC_WORKSPACE_BYTES
    assert L.lib().prism_plan_workspace_bytes(H, nj, N - 1) <= L.PLAN_STATIC_WORKSPACE_BYTES
    r = W.make_request(82, N=1, H=H, nj=nj, dt=dt, kind="smooth")
    P = Projector(H, nj, dt, r.bounds, 1.0, weights="default")
    dev = torch.device("cuda")
    hj = torch.zeros((H, nj), dtype=torch.float32, device=dev)
    outs = _outputs(N, H, nj, dev, 5.0)
    with pytest.raises(PrismError) as e:
        _call(P, None, outs, N, 1, 0, r, hj, hj + 0.5, hj, options(alpha=1.8, tol=1e-3),
              static=True)
    assert e.value.status == L.PRISM_ETOOLARGE
    torch.cuda.synchronize()
    assert float(outs["x"].min()) == 5.0 and float(outs["x"].max()) == 5.0
    assert float(outs["nu"].min()) == 5.0 and int(outs["best"][0]) == -7
    P.close()
