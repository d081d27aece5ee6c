"""Pins of the oracle's primal-update factorization (Sec. III-D, Step 2 and
"Pre-computable factorization")."""

import numpy as np
import pytest

from oracle import factor, problem
import workloads as W


def _rows(H, dt):
    return problem.velocity_unit_rows(H, dt, problem.joint_limits(W.UR5E_BIMANUAL_BOUNDS(1), 0),
                                      0.1, 0.2)


@pytest.mark.parametrize("H,dt,rho", [(2, 0.05, 1.0), (20, 0.05, 1.0), (50, 0.02, 1.0),
                                      (100, 0.02, 1.0), (33, 0.02, 0.1), (17, 0.05, 10.0)])
def test_reduced_inverse_identities(H, dt, rho):
    C = _rows(H, dt).C
    P = factor.penalty_matrix(C, rho)
    K, k = factor.reduced_inverse(P)
    e1 = np.eye(H)[0]
    np.testing.assert_allclose(K, K.T, atol=1e-12)
    np.testing.assert_allclose(K @ e1, 0.0, atol=1e-12)
    assert abs(k[0] - 1.0) < 1e-12
    np.testing.assert_allclose(K @ P, np.eye(H) - np.outer(k, e1), atol=1e-8)
    w = np.linalg.eigvalsh(0.5 * (K + K.T))
    assert w.min() > -1e-12 and w.max() <= 1.0 + 1e-9


@pytest.mark.parametrize("H,dt", [(5, 0.05), (20, 0.05), (50, 0.02)])
def test_lu_solve_satisfies_saddle_system(H, dt):
    """The LU solve returns (x, mu) with P x + mu e1 = r and x_1 = v0, and agrees with K r + k v0."""
    rng = np.random.default_rng(H)
    C = _rows(H, dt).C
    P = factor.penalty_matrix(C, 1.0)
    fac = factor.KKTFactor(P)
    r = rng.normal(0, 3, (H, 7))
    v0 = 0.37
    x, mu = fac.solve_with_multiplier(r, v0)
    e1 = np.eye(H)[:, :1]
    np.testing.assert_allclose(P @ x + e1 * mu[None, :], r, atol=1e-9)
    np.testing.assert_allclose(x[0], v0, atol=1e-12)
    K, k = factor.reduced_inverse(P)
    np.testing.assert_allclose(K @ r + k[:, None] * v0, x, atol=1e-9)


def test_factor_independent_of_boundary_values():
    """Boundary values change only the bounds, never M (Sec. III-D "Boundary value update")."""
    H, dt = 12, 0.05
    lim = problem.joint_limits(W.UR5E_BIMANUAL_BOUNDS(1), 0)
    a = problem.velocity_unit_rows(H, dt, lim, 0.1, 0.2)
    b = problem.velocity_unit_rows(H, dt, lim, -1.0, 1.3)
    np.testing.assert_array_equal(a.C, b.C)
    assert not np.allclose(a.lo, b.lo)
