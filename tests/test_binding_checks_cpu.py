"""The Python binding checks every tensor before its pointer reaches the C ABI,
which cannot check dtype, layout or size: a wrong dtype, a non-contiguous view or a
wrong shape raises ValueError naming the argument, before any library call. Runs on
the CPU: the device check is relaxed so that CPU tensors stand in for device ones."""

import numpy as np
import pytest
import torch

from paper_2608_25666_amd import projector as PJ
from paper_2608_25666_amd import server as SV

H, NJ, N = 10, 3, 8
F32, I32 = torch.float32, torch.int32


@pytest.fixture
def relaxed(monkeypatch):
    monkeypatch.setattr(PJ, "_on_device", lambda t, device: t.device == device)


def _proj():
    P = object.__new__(PJ.Projector)
    P.H, P.nj, P._h = H, NJ, None
    return P


def test_check_rejects_each_kind_of_mismatch():
    t = torch.zeros((N, H, NJ), dtype=F32)
    with pytest.raises(ValueError, match="dtype"):
        PJ._check(t.double(), "a", (N, H, NJ), F32, t.device)
    with pytest.raises(ValueError, match="contiguous"):
        PJ._check(t.transpose(1, 2).contiguous().transpose(1, 2), "a", (N, H, NJ), F32, t.device)
    with pytest.raises(ValueError, match="shape"):
        PJ._check(t[:, :, :2].contiguous(), "a", (N, H, NJ), F32, t.device)
    with pytest.raises(ValueError, match="expected"):
        PJ._check(t, "a", (N, H, NJ), F32, t.device)        # a CPU tensor is not on a GPU
    with pytest.raises(ValueError, match="required"):
        PJ._check(None, "a", (N, H, NJ), F32, t.device, optional=False)
    with pytest.raises(ValueError, match="Tensor"):
        PJ._check(np.zeros((N, H, NJ), np.float32), "a", (N, H, NJ), F32, None)


SOLVE_BAD = {
    "out": torch.zeros((N, H, NJ + 1), dtype=F32),
    "r_primal": torch.zeros((N, NJ), dtype=torch.float64),
    "r_dual": torch.zeros((N + 1, NJ), dtype=F32),
    "iters_out": torch.zeros((N, NJ), dtype=torch.int64),
    "x_warm": torch.zeros((N, NJ, H), dtype=F32),
    "state_warm": torch.zeros((N, NJ, H), dtype=F32),
    "state_out": torch.zeros((N, NJ, 4, H + 1), dtype=F32),
}


@pytest.mark.parametrize("arg", sorted(SOLVE_BAD))
def test_solve_rejects_a_wrong_tensor(relaxed, arg):
    x = torch.zeros((N, H, NJ), dtype=F32)
    with pytest.raises(ValueError, match=arg):
        _proj().solve(x, np.zeros(NJ), np.zeros(NJ), 10, **{arg: SOLVE_BAD[arg]})


def test_solve_rejects_wrong_samples(relaxed):
    with pytest.raises(ValueError, match="samples"):
        _proj().solve(torch.zeros((N, H + 1, NJ), dtype=F32), np.zeros(NJ), np.zeros(NJ), 10)
    with pytest.raises(ValueError, match="samples"):
        _proj().solve(torch.zeros((N, H * NJ), dtype=F32), np.zeros(NJ), np.zeros(NJ), 10)


PLAN_BAD = {
    "samples_out": torch.zeros((N, H, NJ - 1), dtype=F32),
    "r_primal": torch.zeros((N, NJ, 1), dtype=F32),
    "r_dual": torch.zeros((N, NJ), dtype=torch.float16),
    "iters_out": torch.zeros((N, NJ), dtype=F32),
}


@pytest.mark.parametrize("arg", sorted(PLAN_BAD))
def test_plan_step_rejects_a_wrong_tensor(relaxed, arg):
    hj = torch.zeros((H, NJ), dtype=F32)
    with pytest.raises(ValueError, match=arg):
        _proj().plan_step(hj, hj, N, 1, 0, np.zeros(NJ), np.zeros(NJ), hj, 1.0, 0.1, 1.0, 1e-3,
                          10, **{arg: PLAN_BAD[arg]})


@pytest.mark.parametrize("arg", ["nu", "sigma", "theta_ref"])
def test_plan_step_rejects_a_wrong_distribution(relaxed, arg):
    hj = torch.zeros((H, NJ), dtype=F32)
    kw = {"nu": hj, "sigma": hj, "theta_ref": hj}
    kw[arg] = torch.zeros((NJ, H), dtype=F32)
    with pytest.raises(ValueError, match=arg):
        _proj().plan_step(kw["nu"], kw["sigma"], N, 1, 0, np.zeros(NJ), np.zeros(NJ),
                          kw["theta_ref"], 1.0, 0.1, 1.0, 1e-3, 10)


def test_plan_step_rejects_wrong_reused_outputs(relaxed):
    hj = torch.zeros((H, NJ), dtype=F32)
    outs = {"x": torch.zeros((N, H, NJ), dtype=F32), "cost": torch.zeros(N, dtype=torch.float64),
            "omega": torch.zeros(N - 1, dtype=torch.float64), "nu": hj.clone(), "var": hj.clone(),
            "best": torch.zeros(1, dtype=I32)}
    with pytest.raises(ValueError, match="omega"):
        _proj().plan_step(hj, hj, N, 1, 0, np.zeros(NJ), np.zeros(NJ), hj, 1.0, 0.1, 1.0, 1e-3,
                          10, outputs=outs)


def test_literal_and_feasibility_reject_wrong_tensors(relaxed):
    x = torch.zeros((N, H, NJ), dtype=F32)
    with pytest.raises(ValueError, match="x_init"):
        _proj().literal(x, np.zeros(NJ), np.zeros(NJ), 5, x_init=torch.zeros((N, H, NJ + 1)))
    with pytest.raises(ValueError, match="violation"):
        _proj().literal(x, np.zeros(NJ), np.zeros(NJ), 5,
                        violation=torch.zeros((N, NJ), dtype=F32))
    with pytest.raises(ValueError, match="out"):
        _proj().feasibility(x, np.zeros(NJ), np.zeros(NJ),
                            out=torch.zeros((N, NJ, 4), dtype=torch.float64))


def test_batch_rejects_a_wrong_tensor(relaxed):
    B = object.__new__(PJ.Batch)
    B._h = None
    x = torch.zeros((N, H, NJ), dtype=F32)
    req = dict(proj=_proj(), samples=x, q0=np.zeros(NJ), v0=np.zeros(NJ), iters=5,
               state_out=torch.zeros((N, NJ, 4, H - 1), dtype=F32))
    with pytest.raises(ValueError, match="request 0 state_out"):
        B.solve([req])


def test_server_submit_rejects_a_wrong_tensor(relaxed):
    S = object.__new__(SV.Server)
    S._h, S._keep = None, {}
    S._ctrl = {0: _proj()}
    x = torch.zeros((N, H, NJ), dtype=F32)
    with pytest.raises(ValueError, match="iters_out"):
        S.submit(0, x, np.zeros(NJ), np.zeros(NJ), 10, torch.zeros_like(x),
                 iters_out=torch.zeros((N, NJ), dtype=F32))
    with pytest.raises(ValueError, match="out"):
        S.submit(0, x, np.zeros(NJ), np.zeros(NJ), 10, torch.zeros((N, H, NJ), dtype=torch.float64))
