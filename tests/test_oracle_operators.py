"""Pins of the oracle's constraint operators against the paper.

* Each row block of ``problem.physical_rows`` must reproduce positions,
  accelerations and jerks obtained by stepping through time
  (``oracle.feasibility``), Sec. III-D derivative paragraphs.
* Sizes of G, D2 and the jerk stack match the printed dimensions.
* The stacked Kronecker G of eq. (G_h_def) is a row/column permutation of the
  per-joint blocks (joint-wise separability).
* Finite-difference variance factors 2 and 6 (Sec. III-C) hold statistically.
* The white-noise sigma_eff bisection reproduces the printed 0.0045.
"""

import numpy as np
import pytest

from oracle import feasibility, problem
from oracle.sigma_eff import sigma_eff_baseline
from tests.golden.load import read
import workloads as W


def _lim():
    return problem.JointLimits(-2.0, 2.5, -3.0, 3.5, -8.0, 9.0, -60.0, 70.0)


@pytest.mark.parametrize("H,dt", [(2, 0.05), (5, 0.1), (20, 0.05), (37, 0.02)])
def test_rows_match_time_stepping(H, dt):
    rng = np.random.default_rng(H)
    q0, v0 = 0.7, -1.2
    lim = _lim()
    rows = problem.physical_rows(H, dt, lim, q0, v0)
    x = rng.normal(0, 2, H)
    # affine part: lo - c <= C x <= hi - c  ->  C x + c = quantity; recover c from lo
    c = np.concatenate([np.full(H, lim.v_min), np.full(H, lim.q_min), np.full(H, lim.a_min),
                        np.full(H - 1, lim.j_min)]) - rows.lo
    q = rows.C @ x + c
    # time stepping
    pos, acc, jerk = [], [], []
    qk, vprev, aprev = q0, v0, None
    for k in range(H):
        qk = qk + dt * x[k]
        a = (x[k] - vprev) / dt
        pos.append(qk)
        acc.append(a)
        if aprev is not None:
            jerk.append((a - aprev) / dt)
        vprev, aprev = x[k], a
    V, Q, A, J = rows.blocks
    np.testing.assert_allclose(q[V], x, rtol=0, atol=1e-12)
    np.testing.assert_allclose(q[Q], pos, rtol=0, atol=1e-11)
    np.testing.assert_allclose(q[A], acc, rtol=1e-12, atol=1e-9)
    np.testing.assert_allclose(q[J], jerk, rtol=1e-12, atol=1e-7)


def test_violation_module_agrees_with_rows():
    """feasibility.violations (loops) and the row matrices flag the same violations."""
    r = W.white_batch()
    x = r.samples.astype(np.float64)[:8]
    v = feasibility.violations(x, r.dt, r.bounds, r.q0, r.v0)
    for j in range(r.nj):
        lim = problem.joint_limits(r.bounds, j)
        rows = problem.physical_rows(r.H, r.dt, lim, r.q0[j], r.v0[j])
        Cx = x[:, :, j] @ rows.C.T
        viol = np.maximum(Cx - rows.hi, rows.lo - Cx).clip(min=0)
        V, Q, A, J = rows.blocks
        np.testing.assert_allclose(viol[:, V].max(1), v["vel"][:, j], atol=1e-9)
        np.testing.assert_allclose(viol[:, Q].max(1), v["pos"][:, j], atol=1e-9)
        np.testing.assert_allclose(viol[:, A].max(1), v["acc"][:, j], atol=1e-7)
        np.testing.assert_allclose(viol[:, J].max(1), v["jerk"][:, j], atol=1e-5)


@pytest.mark.parametrize("H,nd", [(2, 1), (4, 2), (6, 3), (9, 12)])
def test_printed_dimensions(H, nd):
    d = read("dimensions.txt")
    b = W.UR5E_BIMANUAL_BOUNDS(nd)
    G, h, A, bb = problem.stacked_G_h(H, 0.05, b, np.zeros(nd), np.zeros(nd))
    assert G.shape == ((d["G_rows_per_joint_coeff_H"] * H + d["G_rows_per_joint_const"]) * nd, H * nd)
    assert h.shape == (G.shape[0],)
    assert problem.D2_matrix(H).shape == (d["D2_rows_coeff_H"] * H + d["D2_rows_const"], H)
    assert A.shape == (nd, H * nd) and bb.shape == (nd,)
    # per joint: 4H-1 two-sided rows = (8H-2)/2
    rows = problem.velocity_unit_rows(H, 0.05, problem.joint_limits(b, 0), 0.0, 0.0)
    assert rows.C.shape == (4 * H - 1, H)


@pytest.mark.parametrize("H,nd", [(3, 2), (5, 3)])
def test_kronecker_stack_is_per_joint_blocks(H, nd):
    """Eq. (G_h_def) for N_dof joints equals the per-joint (G_j, h_j) up to ordering."""
    rng = np.random.default_rng(0)
    b = W.Bounds(*[rng.uniform(-3, -1, nd) if i % 2 == 0 else rng.uniform(1, 3, nd)
                   for i in range(8)])
    q0 = rng.uniform(-0.5, 0.5, nd)
    v0 = rng.uniform(-0.5, 0.5, nd)
    dt = 0.05
    G, h, A, bb = problem.stacked_G_h(H, dt, b, q0, v0)
    X = rng.normal(size=(H, nd))           # x[k, j]
    flat = X.reshape(-1)                    # step-major, joint-minor
    stacked_slack = np.sort(h - G @ flat)
    per = []
    for j in range(nd):
        Gj, hj = problem.per_joint_G_h(H, dt, problem.joint_limits(b, j), q0[j], v0[j])
        per.append(hj - Gj @ X[:, j])
    np.testing.assert_allclose(stacked_slack, np.sort(np.concatenate(per)), atol=1e-9)
    np.testing.assert_allclose(A @ flat, X[0], atol=0)
    np.testing.assert_allclose(bb, v0)


def test_velocity_unit_scaling_keeps_feasible_set():
    rng = np.random.default_rng(3)
    H, dt = 12, 0.02
    lim = _lim()
    p = problem.physical_rows(H, dt, lim, 0.3, 0.4)
    s = problem.velocity_unit_rows(H, dt, lim, 0.3, 0.4)
    np.testing.assert_allclose(s.C, np.vstack([np.eye(H), problem.L_matrix(H), problem.D1_matrix(H),
                                               problem.D2_matrix(H)]), atol=1e-12)
    for _ in range(200):
        x = 0.4 + rng.normal(0, 0.05, H)
        fp = np.all((p.C @ x >= p.lo - 1e-12) & (p.C @ x <= p.hi + 1e-12))
        fs = np.all((s.C @ x >= s.lo - 1e-12) & (s.C @ x <= s.hi + 1e-12))
        assert fp == fs


def test_variance_identities():
    """Var(acc) = 2 sigma^2/dt^2 and Var(jerk) = 6 sigma^2/dt^4 on interior rows (Sec. III-C)."""
    d = read("dimensions.txt")
    rng = np.random.default_rng(11)
    H, dt, sigma = 10, 0.05, 0.3
    x = rng.normal(0, sigma, (200_000, H))
    rows = problem.physical_rows(H, dt, _lim(), 0.0, 0.0)
    V, Q, A, J = rows.blocks
    acc = x @ rows.C[A].T
    jerk = x @ rows.C[J].T
    va = acc[:, 1:].var(axis=0)            # interior rows (row 1 has no predecessor sample)
    vj = jerk[:, 1:].var(axis=0)
    np.testing.assert_allclose(va, d["acc_variance_factor"] * sigma ** 2 / dt ** 2, rtol=0.02)
    np.testing.assert_allclose(vj, d["jerk_variance_factor"] * sigma ** 2 / dt ** 4, rtol=0.02)


@pytest.mark.parametrize("H", [10, 15, 20])
def test_sigma_eff_baseline_matches_paper(H):
    g = read("sigma_eff.txt")
    s = sigma_eff_baseline(H, g["dt_assumed"], n=int(g["n_samples"]),
                           threshold=g["violation_threshold"], tol=g["bisection_tol"])
    assert abs(s - g["baseline_sigma_eff"]) <= 0.0004, s
    # a step of 0.05 s would give a four times smaller value: the pin fixes the dt^2 scaling
    s2 = sigma_eff_baseline(H, 0.05, n=50_000)
    assert s2 < 0.5 * g["baseline_sigma_eff"]


def test_sigma_eff_qp_feasible_regime_is_the_identity():
    """Below the baseline's sigma_eff every white-noise sample already meets the bounds,
    so the projection only pins x_1 = v0 and the spread is that of the draws with the
    first step set to v0 (exactly, on the same draws)."""
    from oracle.sigma_eff import sigma_eff_qp
    rng = np.random.Generator(np.random.PCG64(5))
    z = rng.standard_normal((400, 15))
    sigma = 1e-3
    s, x = sigma_eff_qp(z, sigma, 0.1, v0=0.0, tol=1e-12)
    ref = sigma * z.copy()
    ref[:, 0] = 0.0
    np.testing.assert_allclose(x, ref, atol=1e-13)
    assert abs(s - ref.std()) <= 1e-12


def test_sigma_eff_qp_is_bounded_and_grows_with_sigma():
    """Projected velocities lie within |v| <= 1 (so the spread is below 1) and their
    spread grows with the sampling sigma (common draws)."""
    from oracle.sigma_eff import sigma_eff_qp
    rng = np.random.Generator(np.random.PCG64(6))
    z = rng.standard_normal((300, 15))
    prev = 0.0
    for sigma in (0.05, 0.3, 1.0, 3.0):
        s, x = sigma_eff_qp(z, sigma, 0.1, tol=1e-7)
        assert np.abs(x).max() <= 1.0 + 1e-6
        a = np.diff(x, axis=1) / 0.1
        j = np.diff(x, n=2, axis=1) / 0.01
        assert np.abs(a).max() <= 2.0 + 1e-5 and np.abs(j).max() <= 4.0 + 1e-4
        assert s > prev
        prev = s
    assert prev < 1.0
