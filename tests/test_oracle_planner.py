"""Pins of the oracle's optimizer step around the projection (oracle/planner.py):
the counter-based generator against its published known-answer vectors, the
normals' moments, the cost on hand-worked cases, the softmax weights and moment
update on cases that reduce to plain statistics, and the feasibility of the
updated mean (a convex combination of projected samples)."""

import os

import numpy as np
import pytest

from oracle import feasibility, planner
import workloads as W

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = [int(w) for w in planner.philox4x32_10(ctr, key)]
        assert got == out, (ctr, key, [hex(g) for g in got])


def test_philox_vectorised_equals_scalar_calls():
    rng = np.random.default_rng(1)
    c = rng.integers(0, 2 ** 32, size=(4, 50), dtype=np.uint64)
    k = rng.integers(0, 2 ** 32, size=(2,), dtype=np.uint64)
    batch = planner.philox4x32_10([c[0], c[1], c[2], c[3]], [k[0], k[1]])
    for i in (0, 17, 49):
        one = planner.philox4x32_10([int(c[0, i]), int(c[1, i]), int(c[2, i]), int(c[3, i])],
                                    [int(k[0]), int(k[1])])
        assert [int(b[i]) for b in batch] == [int(o) for o in one]


def test_normals_have_standard_moments_and_depend_on_seed_and_stream():
    z = planner.standard_normals((1 << 20,), seed=7, stream=0)
    n = z.size
    assert abs(z.mean()) < 5.0 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.05
    assert abs(np.mean(z > 1.0) - 0.158655) < 0.002          # standard normal tail
    assert np.abs(z).max() < 6.0                               # 23-bit uniforms: |z| <= 5.8
    z2 = planner.standard_normals((1 << 20,), seed=7, stream=1)
    z3 = planner.standard_normals((1 << 20,), seed=8, stream=0)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 0.01 and abs(np.corrcoef(z, z3)[0, 1]) < 0.01
    # element e does not depend on the array's shape (flat row-major index)
    a = planner.standard_normals((4, 5, 6), seed=3, stream=2)
    b = planner.standard_normals((120,), seed=3, stream=2)
    np.testing.assert_array_equal(a.ravel(), b)


def test_tracking_cost_hand_cases():
    # H = 2, one joint: x = (1, 2), q0 = 0, dt = 0.5 -> theta = (0.5, 1.5); ref = 0
    x = np.array([[[1.0], [2.0]]])
    c = planner.tracking_cost(x, [0.0], 0.5, np.zeros((2, 1)), w_pos=3.0, w_vel=0.5)
    assert c.shape == (1,) and abs(c[0] - (3.0 * (0.25 + 2.25) + 0.5 * (1.0 + 4.0))) < 1e-14
    # the reference equal to the integrated positions leaves only the velocity term
    rng = np.random.default_rng(2)
    x = rng.normal(size=(3, 7, 2))
    q0 = np.array([0.3, -1.0])
    ref = q0[None, :] + 0.1 * np.cumsum(x[1], axis=0)
    c = planner.tracking_cost(x, q0, 0.1, ref, w_pos=10.0, w_vel=2.0)
    assert abs(c[1] - 2.0 * np.sum(x[1] ** 2)) < 1e-12
    assert c[0] > 2.0 * np.sum(x[0] ** 2) and c[2] > 2.0 * np.sum(x[2] ** 2)


def test_softmax_weights():
    c = np.array([3.0, 1.0, 2.0, 1.0 + np.log(2.0)])
    w = planner.softmax_weights(c, tau=1.0)
    assert abs(w.sum() - 1.0) < 1e-15
    assert abs(w[1] / w[3] - 2.0) < 1e-12                     # cost gap tau ln 2 -> ratio 2
    assert np.argmax(w) == np.argmin(c)
    np.testing.assert_allclose(planner.softmax_weights(c + 1e4, 1.0), w, rtol=1e-12)
    np.testing.assert_allclose(planner.softmax_weights(c, 1e12), np.full(4, 0.25), rtol=1e-9)
    w_small = planner.softmax_weights(c, 1e-3)
    assert w_small[1] > 0.999                                   # tau -> 0: the best sample


def test_moments_reduce_to_plain_statistics():
    rng = np.random.default_rng(3)
    x = rng.normal(size=(50, 6, 3))
    nu, var = planner.moments(x, np.full(50, 1.0 / 50), eps=1e-4)
    np.testing.assert_allclose(nu, x.mean(axis=0), atol=1e-14)
    np.testing.assert_allclose(var, x.var(axis=0) + 1e-4, atol=1e-13)
    om = np.zeros(50)
    om[17] = 1.0
    nu, var = planner.moments(x, om, eps=1e-3)
    np.testing.assert_array_equal(nu, x[17])
    np.testing.assert_allclose(var, 1e-3, atol=1e-16)


def test_plan_step_updated_mean_is_feasible():
    """Projected samples are feasible and the new mean is their convex combination,
    so it is feasible too (the feasible set is convex)."""
    r = W.make_request(11, N=40, H=15, nj=2, dt=0.05, kind="white")
    nu = np.zeros((15, 2))
    sigma = np.full((15, 2), 1.5)
    ref = np.tile(np.linspace(0.0, 0.5, 15)[:, None], (1, 2)) + r.q0[None, :]
    res = planner.plan_step(nu, sigma, 40, seed=5, stream=0, H=15, dt=0.05, bounds=r.bounds,
                            q0=r.q0, v0=r.v0, theta_ref=ref, w_pos=10.0, w_vel=0.1, tau=1.0,
                            eps=1e-3, iters=20000, alpha=1.6, weights=(1.0, 2.5 / 15, 4.0, 20.0),
                            tol=1e-9, check_every=50)
    assert max(feasibility.max_violation(res.x, 0.05, r.bounds, r.q0, r.v0).values()) < 1e-6
    m = res.nu[None]
    assert max(feasibility.max_violation(m, 0.05, r.bounds, r.q0, r.v0).values()) < 1e-6
    assert abs(res.omega.sum() - 1.0) < 1e-12 and res.best == int(np.argmax(res.omega))
    assert np.all(res.var >= 1e-3)
