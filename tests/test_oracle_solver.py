"""Pins of the oracle's ADMM iteration and of the exact projection.

The exact projection x* (Sec. III-A, eq. (proj_cost)) is pinned by brute-force
face enumeration, KKT certificates, SLSQP, and closed-form special cases. The
ADMM iterates at a fixed count have no printed values; they are pinned by the
optimality conditions of each step and by convergence to x*.
"""

import numpy as np
import pytest
import scipy.optimize

from oracle import admm, exact, factor, problem
import workloads as W


def _lim(tight=True):
    if tight:
        return problem.JointLimits(-0.5, 0.6, -1.5, 1.4, -6.0, 7.0, -50.0, 40.0)
    return problem.JointLimits(-1e6, 1e6, -1e6, 1e6, -1e9, 1e9, -1e12, 1e12)


@pytest.mark.parametrize("H", [2, 3, 4, 5])
def test_admm_converges_to_brute_force(H):
    rng = np.random.default_rng(100 + H)
    dt = 0.05
    lim = _lim()
    for trial in range(4):
        q0 = rng.uniform(-0.3, 0.3)
        v0 = rng.uniform(-1.0, 1.0)
        xt = rng.normal(0.0, 2.5, H)
        rows = problem.velocity_unit_rows(H, dt, lim, q0, v0)
        xb = exact.brute_force(xt, rows.C, rows.lo, rows.hi, v0)
        assert xb is not None
        viol, stat = exact.kkt_certificate(xb, xt, rows.C, rows.lo, rows.hi, v0)
        assert viol < 1e-9 and stat < 1e-9
        res = admm.admm_joint(xt[None, :], H, dt, lim, q0, v0, iters=30000, tol=1e-11,
                              check_every=50)
        np.testing.assert_allclose(res.x[0], xb, atol=1e-8)
        xs = exact.slsqp(xt, rows.C, rows.lo, rows.hi, v0)
        np.testing.assert_allclose(xs, xb, atol=1e-6)


def test_certificate_rejects_wrong_points():
    """A perturbed optimum fails the certificate (the check is not vacuous)."""
    rng = np.random.default_rng(5)
    H, dt = 5, 0.05
    lim = _lim()
    xt = rng.normal(0, 2.5, H)
    rows = problem.velocity_unit_rows(H, dt, lim, 0.1, 0.3)
    xb = exact.brute_force(xt, rows.C, rows.lo, rows.hi, 0.3)
    for k in range(1, H):
        for eps in (1e-3, -1e-3):
            x = xb.copy()
            x[k] += eps
            viol, stat = exact.kkt_certificate(x, xt, rows.C, rows.lo, rows.hi, 0.3, act_tol=1e-9)
            assert viol > 1e-6 or stat > 1e-6


@pytest.mark.parametrize("H,dt,N", [(20, 0.05, 24), (50, 0.02, 12)])
def test_admm_converges_to_certified_projection(H, dt, N):
    """At realistic sizes the converged iterate, polished on its active set, passes KKT."""
    r = W.make_request(7, N=N, H=H, nj=2, dt=dt, kind="smooth" if H == 50 else "white")
    for j in range(2):
        lim = problem.joint_limits(r.bounds, j)
        rows = problem.velocity_unit_rows(H, dt, lim, r.q0[j], r.v0[j])
        res = admm.admm_joint(r.samples[:, :, j], H, dt, lim, r.q0[j], r.v0[j], iters=40000,
                              tol=1e-10, check_every=100, alpha=1.6)
        for c in range(N):
            xt = r.samples[c, :, j].astype(np.float64)
            xp = exact.polish(xt, rows.C, rows.lo, rows.hi, r.v0[j], res.y[c])
            viol, stat = exact.kkt_certificate(xp, xt, rows.C, rows.lo, rows.hi, r.v0[j])
            assert viol < 1e-8 and stat < 1e-8, (c, viol, stat)
            np.testing.assert_allclose(res.x[c], xp, atol=1e-7)


def test_loose_bounds_return_sample_with_boundary_velocity():
    """All bounds inactive: x* = x~ with x_1 := v0 (closed form)."""
    rng = np.random.default_rng(1)
    H, dt = 15, 0.05
    xt = rng.normal(0, 1, (9, H))
    res = admm.admm_joint(xt, H, dt, _lim(False), 0.0, 0.25, iters=50)
    want = xt.copy()
    want[:, 0] = 0.25
    np.testing.assert_allclose(res.x, want, atol=1e-12)


def test_velocity_only_bounds_clip():
    """Only velocity bounds finite: x*_k = clip(x~_k) for k >= 2, x*_1 = v0."""
    rng = np.random.default_rng(2)
    H, dt = 12, 0.05
    lim = problem.JointLimits(-1e6, 1e6, -0.7, 0.9, -1e9, 1e9, -1e12, 1e12)
    xt = rng.normal(0, 1.5, (10, H))
    res = admm.admm_joint(xt, H, dt, lim, 0.0, 0.1, iters=3000, tol=1e-12, check_every=10)
    want = np.clip(xt, -0.7, 0.9)
    want[:, 0] = 0.1
    np.testing.assert_allclose(res.x, want, atol=1e-9)


def test_feasible_input_returned_unchanged():
    """A feasible sample with x~_1 = v0 is a fixed point from the first iterate on.

    The oracle's primal step is an LU solve of M, so it returns the input to
    rounding; the library's incremental form keeps it bit for bit."""
    H, dt = 20, 0.05
    lim = problem.joint_limits(W.UR5E_BIMANUAL_BOUNDS(1), 0)
    t = np.arange(1, H + 1) * dt
    xt = np.stack([0.3 + 0.2 * np.sin(2 * np.pi * 0.5 * t + p) for p in (0.0, 0.4, 1.0)])
    xt[:, 0] = 0.3 + 0.2 * np.sin(2 * np.pi * 0.5 * dt + np.array([0.0, 0.4, 1.0]))
    for c in range(3):
        v0 = xt[c, 0]
        rows = problem.velocity_unit_rows(H, dt, lim, 0.0, v0)
        s = rows.C @ xt[c]
        assert np.all((s >= rows.lo) & (s <= rows.hi))
        res = admm.admm_joint(xt[c:c + 1], H, dt, lim, 0.0, v0, iters=100)
        np.testing.assert_allclose(res.x[0], xt[c], rtol=0, atol=1e-12)


def test_primal_step_solves_its_subproblem():
    """After one iteration x solves min 1/2||x-x~||^2 + rho/2||Cx - z0 + y0/rho||^2, x_1 = v0,
    with z0 = clip(C x0) and y0 = rho (C x0 - z0) from the first slack/multiplier pass."""
    rng = np.random.default_rng(4)
    H, dt, rho, v0 = 20, 0.05, 1.7, 0.4
    lim = _lim()
    rows = problem.velocity_unit_rows(H, dt, lim, 0.05, v0)
    xt = rng.normal(0, 2, (3, H))
    x0 = xt.copy()
    x0[:, 0] = v0
    s0 = x0 @ rows.C.T
    z0 = np.clip(s0, rows.lo, rows.hi)
    u0 = s0 - z0                                                 # y0 / rho
    res = admm.admm_joint(xt, H, dt, lim, 0.05, v0, rho=rho, iters=1)
    x1 = res.x
    grad = (x1 - xt) + rho * (x1 @ rows.C.T - z0 + u0) @ rows.C
    np.testing.assert_allclose(grad[:, 1:], 0.0, atol=1e-9)    # row 1 absorbed by mu
    np.testing.assert_allclose(x1[:, 0], v0, atol=0)
    # z-step and y-step consistency: z in the box, y sign pattern of the normal cone
    z, y = res.z, res.y
    assert np.all(z >= rows.lo - 1e-12) and np.all(z <= rows.hi + 1e-12)
    interior = (z > rows.lo + 1e-9) & (z < rows.hi - 1e-9)
    np.testing.assert_allclose(y[interior], 0.0, atol=1e-9)
    assert np.all(y[np.isclose(z, rows.hi)] >= -1e-12)
    assert np.all(y[np.isclose(z, rows.lo)] <= 1e-12)


def test_dual_residual_identity():
    """With alpha = 1, r_d equals rho ||C^T (z^L - z^{L-1})|| on rows 2..H."""
    r = W.white_batch()
    j = 3
    lim = problem.joint_limits(r.bounds, j)
    rows = problem.velocity_unit_rows(r.H, r.dt, lim, r.q0[j], r.v0[j])
    a = admm.admm_joint(r.samples[:8, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], iters=29)
    b = admm.admm_joint(r.samples[:8, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], iters=30)
    direct = np.max(np.abs((b.z - a.z) @ rows.C)[:, 1:], axis=1)
    np.testing.assert_allclose(b.r_d, direct, rtol=1e-6, atol=1e-9)


def test_projection_properties():
    """Idempotence P(P(x)) = P(x) and non-expansiveness ||P(a)-P(b)|| <= ||a-b||."""
    rng = np.random.default_rng(9)
    H, dt = 10, 0.05
    lim = _lim()
    q0, v0 = 0.1, 0.2
    a = rng.normal(0, 2, (6, H))
    b = a + rng.normal(0, 0.5, (6, H))
    kw = dict(iters=60000, tol=1e-11, check_every=100, alpha=1.6)
    pa = admm.admm_joint(a, H, dt, lim, q0, v0, **kw).x
    pb = admm.admm_joint(b, H, dt, lim, q0, v0, **kw).x
    ppa = admm.admm_joint(pa, H, dt, lim, q0, v0, **kw).x
    np.testing.assert_allclose(ppa, pa, atol=1e-8)
    assert np.all(np.linalg.norm(pa - pb, axis=1) <= np.linalg.norm(a - b, axis=1) + 1e-8)


def test_joint_separability_against_stacked_problem():
    """Per-joint solutions certify as optimal for the stacked eq. (compact_qp) (Sec. III-D)."""
    r = W.make_request(3, N=2, H=6, nj=3, dt=0.05, kind="white", sigma=2.0)
    res = admm.solve_request(r.samples, r.H, r.dt, r.bounds, r.q0, r.v0, iters=60000,
                             tol=1e-11, check_every=100, alpha=1.6)
    G, h, A, b = problem.stacked_G_h(r.H, r.dt, r.bounds, r.q0, r.v0)
    for s in range(r.N):
        xt = r.samples[s].astype(np.float64).reshape(-1)
        x = res.x[s].reshape(-1)
        Gx = G @ x
        assert np.max(Gx - h) < 1e-8
        act = np.where(Gx >= h - 1e-7)[0]
        # stationarity: x - xt + G_act^T lam + A^T mu = 0, lam >= 0
        B = np.hstack([G[act].T, A.T, -A.T])
        w, _ = scipy.optimize.nnls(B, xt - x)
        assert np.max(np.abs(B @ w - (xt - x))) < 1e-7


def test_per_column_early_exit():
    """Each column stops at the first check point where its own max(r_p, r_d) <= tol:
    its count is a check point, the residual meets tol there, and a fixed-count run one
    check period shorter leaves that column above tol. A run with per-column counts
    equal to the stops reproduces the early-exit iterates bit for bit."""
    r = W.white_batch()
    tol, ce = 1e-3, 10
    res = admm.solve_request(r.samples[:40], r.H, r.dt, r.bounds, r.q0, r.v0, iters=5000,
                             tol=tol, check_every=ce)
    assert np.all(res.iters % ce == 0)
    assert np.all(np.maximum(res.r_p, res.r_d) <= tol)
    assert len(np.unique(res.iters)) > 5          # columns of one joint stop apart
    fixed = admm.solve_request(r.samples[:40], r.H, r.dt, r.bounds, r.q0, r.v0,
                               iters=res.iters)
    np.testing.assert_array_equal(fixed.x, res.x)
    np.testing.assert_array_equal(fixed.iters, res.iters)
    before = admm.solve_request(r.samples[:40], r.H, r.dt, r.bounds, r.q0, r.v0,
                                iters=np.maximum(res.iters - ce, 0))
    late = np.maximum(before.r_p, before.r_d)
    assert np.all(late[res.iters > 0] > tol)


def test_per_column_counts_equal_separate_runs():
    """Column c of a run with counts iters[c] equals a run of that column alone (to BLAS
    rounding, which depends on how many columns share a product)."""
    r = W.make_request(8, N=5, H=12, nj=1, dt=0.05, kind="white", sigma=1.5)
    lim = problem.joint_limits(r.bounds, 0)
    counts = np.array([0, 1, 7, 30, 12])
    kw = dict(alpha=1.8, weights=(1.7, 2.125 / 12, 13.6, 17.0))
    a = admm.admm_joint(r.samples[:, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0], iters=counts, **kw)
    for c, n in enumerate(counts):
        b = admm.admm_joint(r.samples[c:c + 1, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0],
                            iters=int(n), **kw)
        np.testing.assert_allclose(a.x[c], b.x[0], rtol=0, atol=1e-12)
        np.testing.assert_allclose(a.y[c], b.y[0], rtol=0, atol=1e-11)
    assert np.all(a.iters == counts)


def test_warm_start_at_solution_is_fixed_point():
    r = W.make_request(2, N=4, H=12, nj=1, dt=0.05, kind="white", sigma=2.0)
    lim = problem.joint_limits(r.bounds, 0)
    kw = dict(iters=40000, tol=1e-12, check_every=100)
    res = admm.admm_joint(r.samples[:, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0], **kw)
    again = admm.admm_joint(r.samples[:, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0], iters=20,
                            warm_x=res.x, warm_y=res.y)
    np.testing.assert_allclose(again.x, res.x, atol=1e-9)


def test_literal_iteration_stops_at_any_feasible_point():
    """As printed, every feasible x paired with lambda = x - x~ is a fixed point, so the
    iteration settles on a feasible point that need not be x* (documents the reading of
    the "ADMM Solver" passage; the headline iteration carries y in constraint space)."""
    rng = np.random.default_rng(12)
    H, dt = 10, 0.05
    lim = _lim()
    q0, v0 = 0.0, 0.2
    xt = rng.normal(0, 2, (4, H))
    feasible = np.full((4, H), v0)          # constant velocity: feasible for these limits
    xl, viol = admm.literal_joint(xt, H, dt, lim, q0, v0, delta=1.0, iters=300,
                                  x_init=feasible, lam_init=feasible - xt)
    np.testing.assert_allclose(xl, feasible, atol=1e-9)
    xstar = admm.admm_joint(xt, H, dt, lim, q0, v0, iters=40000, tol=1e-11, check_every=100).x
    assert np.max(np.abs(feasible - xstar)) > 0.1
    # from the sample itself the printed iteration reaches a feasible point, not x*
    xl2, viol2 = admm.literal_joint(xt, H, dt, lim, q0, v0, delta=1.0, iters=5000)
    assert np.all(viol2 < 1e-3)
    assert np.max(np.abs(xl2 - xstar)) > 1e-2


def test_kkt_factor_route_equals_reduced_inverse_route():
    """Iterating with x = K r + k v0 gives the same iterates as the LU solve of M."""
    r = W.white_batch()
    j = 0
    lim = problem.joint_limits(r.bounds, j)
    rows = problem.velocity_unit_rows(r.H, r.dt, lim, r.q0[j], r.v0[j])
    K, k = factor.reduced_inverse(factor.penalty_matrix(rows.C, 1.0))
    xt = r.samples[:5, :, j].astype(np.float64).T
    x = xt.copy()
    x[0] = r.v0[j]
    s0 = rows.C @ x
    z = np.clip(s0, rows.lo[:, None], rows.hi[:, None])
    y = s0 - z
    for _ in range(50):
        x = K @ (xt + rows.C.T @ (z - y)) + k[:, None] * r.v0[j]
        s = rows.C @ x
        zn = np.clip(s + y, rows.lo[:, None], rows.hi[:, None])
        y = y + s - zn
        z = zn
    res = admm.admm_joint(r.samples[:5, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], iters=50)
    np.testing.assert_allclose(res.x, x.T, atol=1e-10)


W_ACCEL = (1.0, 0.125, 4.0, 20.0)   # block weights (velocity, position, acceleration, jerk)


def test_block_weights_keep_the_fixed_point():
    """A diagonal block penalty changes the path, not the limit: the converged iterate
    passes the KKT certificate and equals the unit-weight limit."""
    r = W.make_request(31, N=12, H=20, nj=2, dt=0.05, kind="white", sigma=1.0)
    for j in range(2):
        lim = problem.joint_limits(r.bounds, j)
        rows = problem.velocity_unit_rows(r.H, r.dt, lim, r.q0[j], r.v0[j])
        a = admm.admm_joint(r.samples[:, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], alpha=1.6,
                            iters=60000, tol=1e-11, check_every=50, weights=W_ACCEL)
        b = admm.admm_joint(r.samples[:, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], alpha=1.6,
                            iters=60000, tol=1e-11, check_every=50)
        np.testing.assert_allclose(a.x, b.x, atol=1e-7)
        for c in range(r.N):
            xt = r.samples[c, :, j].astype(np.float64)
            xp = exact.polish(xt, rows.C, rows.lo, rows.hi, r.v0[j], a.y[c])
            viol, stat = exact.kkt_certificate(xp, xt, rows.C, rows.lo, rows.hi, r.v0[j])
            assert viol < 1e-8 and stat < 1e-8


def test_block_weighted_primal_step_solves_its_subproblem():
    """With R = rho diag(w): x1 minimises 1/2||x-x~||^2 + 1/2||Cx - z0 + R^-1 y0||_R^2, x_1 = v0."""
    rng = np.random.default_rng(41)
    H, dt, rho, v0 = 18, 0.05, 1.3, 0.2
    lim = _lim()
    rows = problem.velocity_unit_rows(H, dt, lim, 0.0, v0)
    R = admm.block_penalty(H, rho, W_ACCEL)
    xt = rng.normal(0, 2, (3, H))
    x0 = xt.copy()
    x0[:, 0] = v0
    s0 = x0 @ rows.C.T
    z0 = np.clip(s0, rows.lo, rows.hi)
    u0 = s0 - z0                                   # R^-1 y0
    res = admm.admm_joint(xt, H, dt, lim, 0.0, v0, rho=rho, iters=1, weights=W_ACCEL)
    x1 = res.x
    grad = (x1 - xt) + ((x1 @ rows.C.T - z0 + u0) * R) @ rows.C
    np.testing.assert_allclose(grad[:, 1:], 0.0, atol=1e-9)
    np.testing.assert_allclose(res.x[:, 0], v0, atol=1e-14)


def test_block_weighted_dual_residual_identity():
    """alpha = 1: r_d = ||C^T R (z^L - z^{L-1})|| on rows 2..H with the block penalty."""
    r = W.white_batch()
    j = 2
    lim = problem.joint_limits(r.bounds, j)
    rows = problem.velocity_unit_rows(r.H, r.dt, lim, r.q0[j], r.v0[j])
    R = admm.block_penalty(r.H, 1.0, W_ACCEL)
    a = admm.admm_joint(r.samples[:8, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], iters=29,
                        weights=W_ACCEL)
    b = admm.admm_joint(r.samples[:8, :, j], r.H, r.dt, lim, r.q0[j], r.v0[j], iters=30,
                        weights=W_ACCEL)
    direct = np.max(np.abs(((b.z - a.z) * R) @ rows.C)[:, 1:], axis=1)
    np.testing.assert_allclose(b.r_d, direct, rtol=1e-6, atol=1e-9)


def test_warm_start_with_slack_at_solution_is_fixed_point():
    """With the previous slack carried along, a converged state (x*, z*, y*) is a fixed
    point of the warm restart for relaxation alpha != 1 as well: C x* = z*, so the
    relaxed step reproduces z*, and y* lies in the normal cone of the box at z*."""
    r = W.make_request(5, N=6, H=14, nj=1, dt=0.05, kind="white", sigma=1.5)
    lim = problem.joint_limits(r.bounds, 0)
    kw = dict(alpha=1.6, weights=W_ACCEL)
    a = admm.admm_joint(r.samples[:, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0], iters=60000,
                        tol=1e-12, check_every=100, **kw)
    b = admm.admm_joint(r.samples[:, :, 0], r.H, r.dt, lim, r.q0[0], r.v0[0], iters=25,
                        warm_x=a.x, warm_y=a.y, warm_z=a.z, **kw)
    np.testing.assert_allclose(b.x, a.x, atol=1e-9)
    np.testing.assert_allclose(b.y, a.y, atol=1e-8)


def test_advance_warm_start_hand_example():
    """H = 3, one column, values worked by hand: x = (0.5, 1, 2) has C x =
    V (0.5, 1, 2) | Q (0.5, 1.5, 3.5) | A (0.5, 0.5, 1) | J (0, 0.5); the slack
    deviates from it by d = 0.1 * (1..11). With v0_new = -0.25 the shifted iterate
    (-0.25, 2, 2) has C x' = V (-0.25, 2, 2) | Q (-0.25, 1.75, 3.75) |
    A (-0.25, 2.25, 0) | J (2.5, -2.25), and the shifted deviation is
    V (.2, .3, .3) | Q (.5, .6, .6) | A (0, .9, .9) | J (1.1, 1.1)."""
    H = 3
    x = np.array([0.5, 1.0, 2.0]).reshape(1, 3, 1)
    Cx = np.array([0.5, 1, 2, 0.5, 1.5, 3.5, 0.5, 0.5, 1.0, 0.0, 0.5])
    y = np.arange(1.0, 12.0).reshape(1, 1, 11)
    z = (Cx + 0.1 * np.arange(1.0, 12.0)).reshape(1, 1, 11)
    xs, ys, zs = admm.advance_warm_start(x, y, z, H, [-0.25])
    np.testing.assert_array_equal(xs[0, :, 0], [-0.25, 2.0, 2.0])
    np.testing.assert_array_equal(ys[0, 0], [2, 3, 3, 5, 6, 6, 0, 9, 9, 11, 11])
    np.testing.assert_allclose(zs[0, 0], [-0.05, 2.3, 2.3, 0.25, 2.35, 4.35, -0.25, 3.15, 0.9,
                                          3.6, -1.15], atol=1e-12)


@pytest.mark.parametrize("alpha", [1.0, 1.6])
def test_advance_warm_start_keeps_a_stationary_solution(alpha):
    """Samples above the velocity limit and v0 at the limit: the projection is the
    constant trajectory x = v_max with active velocity rows. Time-shifting changes
    nothing, so the advanced state of the converged solve must pass the first residual
    check of the next solve (iteration 0) -- which fails if any block's offset is off."""
    H, vmax = 12, 1.4
    lim = problem.JointLimits(-1e6, 1e6, -1.5, vmax, -7.0, 7.0, -50.0, 50.0)
    xt = np.full((5, H), 2.0)
    kw = dict(alpha=alpha, weights=(1.0, 0.2, 4.0, 20.0))
    a = admm.admm_joint(xt, H, 0.05, lim, 0.1, vmax, iters=60000, tol=1e-12, check_every=50, **kw)
    np.testing.assert_allclose(a.x, vmax, atol=1e-9)
    xs, ys, zs = admm.advance_warm_start(a.x[:, :, None], a.y[:, None, :], a.z[:, None, :], H,
                                         [vmax])
    b = admm.admm_joint(xt, H, 0.05, lim, 0.1, vmax, iters=100, tol=1e-8, check_every=10,
                        warm_x=xs[:, :, 0], warm_y=ys[:, 0], warm_z=zs[:, 0], **kw)
    assert np.all(b.iters == 0)
    np.testing.assert_allclose(b.x, a.x, atol=1e-9)


def _aug_lag(x, xt, lam, zeta, G, h, delta):
    """Eq. (aug_lag) as a scalar, one column."""
    r = G @ x - h + zeta
    return 0.5 * np.sum((x - xt) ** 2) - lam @ x + 0.5 * delta * (r @ r)


@pytest.mark.parametrize("delta", [1.0, 0.05])
def test_literal_primal_step_minimizes_the_augmented_objective(delta):
    """One printed pass from (x~ with x_1 := v0, lambda = 0): the returned x has x_1 = v0
    and zero gradient of the scalar eq. (aug_lag) in every free step (central
    differences, exact for a quadratic up to rounding), with zeta = max(0, h - G x0)."""
    rng = np.random.default_rng(31)
    H, dt = 7, 0.05
    lim = _lim()
    q0, v0 = 0.1, 0.3
    xt = rng.normal(0, 2, (3, H))
    x1, _, lam1 = admm.literal_joint(xt, H, dt, lim, q0, v0, delta=delta, iters=1,
                                     return_lam=True)
    G, h = problem.per_joint_G_h(H, dt, lim, q0, v0)
    for c in range(3):
        x0 = xt[c].copy()
        x0[0] = v0
        zeta = np.maximum(0.0, h - G @ x0)
        assert abs(x1[c, 0] - v0) <= 1e-12
        scale = 1.0 + delta * np.abs(G).max() ** 2 * np.abs(x1[c]).max()
        for k in range(1, H):
            e = np.zeros(H)
            e[k] = 1e-3
            gk = (_aug_lag(x1[c] + e, xt[c], np.zeros(H), zeta, G, h, delta)
                  - _aug_lag(x1[c] - e, xt[c], np.zeros(H), zeta, G, h, delta)) / 2e-3
            assert abs(gk) <= 1e-7 * scale, (c, k, gk)


def test_literal_multiplier_step_closed_form():
    """With the dual step delta/2 of eq. (admm_dual) and an exact primal step, the
    stationarity of Step 2 turns Step 3 into lambda' = (lambda + x' - x~) / 2 on every
    free step (steps 2..H): a closed form that a wrong dual step size or sign breaks."""
    rng = np.random.default_rng(32)
    H, dt = 9, 0.05
    lim = _lim()
    q0, v0 = -0.1, -0.2
    xt = rng.normal(0, 2, (4, H))
    lam0 = rng.normal(0, 0.5, (4, H))
    for delta in (1.0, 0.3):
        x1, _, lam1 = admm.literal_joint(xt, H, dt, lim, q0, v0, delta=delta, iters=1,
                                         lam_init=lam0, return_lam=True)
        want = 0.5 * (lam0 + x1 - xt)
        np.testing.assert_allclose(lam1[:, 1:], want[:, 1:], atol=1e-7, rtol=1e-9)


def test_literal_feasible_sample_is_a_fixed_point():
    """A feasible sample with x~_1 = v0 has zeta = h - G x~, so the primal step returns it
    and the multiplier stays zero: unchanged after any number of passes."""
    H, dt = 12, 0.05
    lim = _lim()
    q0, v0 = 0.0, 0.2
    xt = np.stack([np.full(H, v0), v0 + 0.01 * np.sin(np.arange(H))])
    xt[:, 0] = v0
    G, h = problem.per_joint_G_h(H, dt, lim, q0, v0)
    assert np.all(G @ xt.T <= h[:, None])
    x, viol = admm.literal_joint(xt, H, dt, lim, q0, v0, delta=1.0, iters=50)
    np.testing.assert_allclose(x, xt, atol=1e-12)
    assert np.all(viol == 0.0)


# ---------------------------------------------------------------------------
# The over-relaxed step (alpha != 1) as the benchmarks run it
# ---------------------------------------------------------------------------

ALPHA = 1.8


def _default_weights(H):
    return (1.7, 2.125 / H, 13.6, 17.0)


def _row_penalty(H, rho, w):
    """R written out per row: velocity, position, acceleration rows (H each), jerk (H-1)."""
    return np.concatenate([np.full(H, rho * w[0]), np.full(H, rho * w[1]),
                           np.full(H, rho * w[2]), np.full(H - 1, rho * w[3])])


def _single_state_iterates(xt, C, lo, hi, Rv, v0, alpha, counts):
    """The iteration in its single-state form, written independently of the oracle and in
    dense FP64: one state per constraint row, q = (1 - alpha) z + R^-1 y, and an
    incremental primal step through the inverse of the bordered KKT matrix
    [[I + C^T R C, e1], [e1^T, 0]]:
        t = alpha C x + q,  z = clip(t),  q' = t - alpha z,
        d = (x~ - x) + C^T R (2 z - t - C x),  x' = x + K d.
    Cold start q = (1 - alpha) C x0 with x0 = x~, x0_1 := v0. Returns {L: (x_L, q_L)}
    for every L in counts (x: (ncols, H), q: (ncols, rows))."""
    H = C.shape[1]
    M = np.zeros((H + 1, H + 1))
    M[:H, :H] = np.eye(H) + C.T @ (Rv[:, None] * C)
    M[0, H] = M[H, 0] = 1.0
    K = np.linalg.inv(M)[:H, :H]
    x = np.array(xt, dtype=np.float64)
    x[:, 0] = v0
    q = (1.0 - alpha) * (x @ C.T)
    out = {}
    for L in range(max(counts) + 1):
        s = x @ C.T
        t = alpha * s + q
        z = np.clip(t, lo, hi)
        q = t - alpha * z
        if L in counts:
            out[L] = (x.copy(), q.copy())
        d = (xt - x) + ((2.0 * z - t - s) * Rv) @ C
        x = x + d @ K.T
    return out


def _relaxed_step_violations(alpha=ALPHA, H=20, dt=0.05, rho=1.0, seed=44):
    """Largest violation of each defining property of one relaxed step, taken after
    L iterations (z != C x and y != 0 by then):
      grad   x+ minimises 1/2||x - x~||^2 + 1/2||C x - z + R^-1 y||_R^2 with x_1 = v0
             (zero gradient on steps 2..H, x+_1 = v0);
      box    z+ inside [lo, hi];
      cone   y+ in the normal cone of the box at z+ (0 inside, >= 0 at hi, <= 0 at lo);
      prox   z+ + R^-1 y+ = s^ + R^-1 y with s^ = alpha C x+ + (1 - alpha) z, so that
             (box, cone, prox) make z+ the projection of s^ + R^-1 y onto the box;
      chain  x after L = 1, 2, 5, 30 iterations equals the single-state recurrence."""
    rng = np.random.default_rng(seed)
    lim = _lim()
    q0, v0 = 0.05, 0.4
    w = _default_weights(H)
    rows = problem.velocity_unit_rows(H, dt, lim, q0, v0)
    C, lo, hi = rows.C, rows.lo, rows.hi
    Rv = _row_penalty(H, rho, w)
    xt = rng.normal(0, 2, (4, H))
    kw = dict(rho=rho, alpha=alpha, weights=w)
    v = {}
    for L in (3, 11):
        a = admm.admm_joint(xt, H, dt, lim, q0, v0, iters=L, **kw)
        b = admm.admm_joint(xt, H, dt, lim, q0, v0, iters=L + 1, **kw)
        x1, z0, y0, z1, y1 = b.x, a.z, a.y, b.z, b.y
        grad = (x1 - xt) + ((x1 @ C.T - z0) * Rv + y0) @ C
        v["grad"] = max(v.get("grad", 0.0), np.abs(grad[:, 1:]).max(), np.abs(x1[:, 0] - v0).max())
        v["box"] = max(v.get("box", 0.0), np.maximum(lo - z1, 0).max(), np.maximum(z1 - hi, 0).max())
        inside = (z1 > lo + 1e-9) & (z1 < hi - 1e-9)
        at_hi = np.isclose(z1, hi, rtol=0, atol=1e-9)
        at_lo = np.isclose(z1, lo, rtol=0, atol=1e-9)
        cone = np.concatenate([np.abs(y1[inside]), np.maximum(-y1[at_hi & ~at_lo], 0),
                               np.maximum(y1[at_lo & ~at_hi], 0), [0.0]])
        v["cone"] = max(v.get("cone", 0.0), cone.max())
        shat = alpha * (x1 @ C.T) + (1.0 - alpha) * z0
        v["prox"] = max(v.get("prox", 0.0), np.abs(z1 + y1 / Rv - (shat + y0 / Rv)).max())
    counts = (1, 2, 5, 30)
    ref = _single_state_iterates(xt, C, lo, hi, Rv, v0, alpha, counts)
    chain = 0.0
    for L in counts:
        o = admm.admm_joint(xt, H, dt, lim, q0, v0, iters=L, **kw)
        chain = max(chain, np.abs(o.x - ref[L][0]).max())
        q = (1.0 - alpha) * o.z + o.y / Rv
        chain = max(chain, np.abs(q - ref[L][1]).max())
    v["chain"] = chain
    return v


@pytest.mark.parametrize("alpha", [ALPHA, 1.0, 1.5])
def test_relaxed_step_defining_properties(alpha):
    """alpha = 1.8 (the benchmarks'), the default block weights: each step satisfies the
    optimality conditions of its two subproblems and the iterates equal an independently
    written single-state recurrence."""
    v = _relaxed_step_violations(alpha=alpha)
    print({k: f"{x:.1e}" for k, x in v.items()})
    for k, x in v.items():
        assert x <= 1e-9, (k, x)


def _mut_y_from_s(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: the multiplier step uses s = C x+ instead of the relaxed s^."""
    x = fac.solve(xt + C.T @ (R * z - y), v0)
    s = C @ x
    shat = alpha * s + (1.0 - alpha) * z
    zn = np.clip(shat + y / R, lo, hi)
    return x, zn, y + R * (s - zn)


def _mut_z_from_s(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: the slack step projects s + R^-1 y instead of s^ + R^-1 y."""
    x = fac.solve(xt + C.T @ (R * z - y), v0)
    s = C @ x
    shat = alpha * s + (1.0 - alpha) * z
    zn = np.clip(s + y / R, lo, hi)
    return x, zn, y + R * (shat - zn)


def _mut_no_relaxation(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: alpha ignored (s^ = s in both steps)."""
    x = fac.solve(xt + C.T @ (R * z - y), v0)
    s = C @ x
    zn = np.clip(s + y / R, lo, hi)
    return x, zn, y + R * (s - zn)


def _mut_relaxation_sign(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: s^ = alpha s - (1 - alpha) z."""
    x = fac.solve(xt + C.T @ (R * z - y), v0)
    shat = alpha * (C @ x) - (1.0 - alpha) * z
    zn = np.clip(shat + y / R, lo, hi)
    return x, zn, y + R * (shat - zn)


def _mut_unscaled_multiplier(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: the slack step adds y instead of R^-1 y."""
    x = fac.solve(xt + C.T @ (R * z - y), v0)
    shat = alpha * (C @ x) + (1.0 - alpha) * z
    zn = np.clip(shat + y, lo, hi)
    return x, zn, y + R * (shat - zn)


def _mut_relaxed_primal_rhs(xt, z, y, C, lo, hi, R, fac, v0, alpha):
    """Planted mistake: the primal right-hand side uses C^T (R z + y)."""
    x = fac.solve(xt + C.T @ (R * z + y), v0)
    shat = alpha * (C @ x) + (1.0 - alpha) * z
    zn = np.clip(shat + y / R, lo, hi)
    return x, zn, y + R * (shat - zn)


@pytest.mark.parametrize("mutant", [_mut_y_from_s, _mut_z_from_s, _mut_no_relaxation,
                                    _mut_relaxation_sign, _mut_unscaled_multiplier,
                                    _mut_relaxed_primal_rhs])
def test_relaxed_step_pins_reject_planted_mistakes(monkeypatch, mutant):
    """Each plausible mistake in the oracle's relaxed step, planted in the oracle, breaks
    at least one pin of test_relaxed_step_defining_properties at alpha = 1.8."""
    monkeypatch.setattr(admm, "relaxed_step", mutant)
    v = _relaxed_step_violations(alpha=ALPHA)
    print(mutant.__name__, {k: f"{x:.1e}" for k, x in v.items()})
    assert max(v.values()) > 1e-3
