"""Single-joint sampling diagnostic of Sec. III-C ("Empirical Validation").

Test infrastructure only (see ``oracle/__init__``).

For white-noise velocity samples N(0, sigma^2 I) over a horizon, the paper
defines sigma_eff as the largest sigma whose violation rate (fraction of
trajectories that break any bound at any step) stays below 0.3%, found by a
bisection that stops when the interval is narrower than 1e-4. Bounds:
|v| <= 1 rad/s, |a| <= 2 rad/s^2, |j| <= 4 rad/s^3; accelerations and jerks by
first and second finite differences of the sampled velocities.

The paper prints sigma_eff = 0.0045 for this baseline but does not state the
step or the horizon; its simulation step is 0.1 s (Sec. V-A).
The bisection here reuses one set of standard-normal draws scaled by sigma
(common random numbers), which makes the violation rate monotone in sigma.
"""

from __future__ import annotations

import numpy as np

from . import problem


def violation_rate(z: np.ndarray, sigma: float, dt: float, v_max=1.0, a_max=2.0, j_max=4.0):
    """Fraction of rows of sigma*z (shape [n, H]) that violate any bound.

    Accelerations and jerks use the operator rows of eqs. (acc_stack) and
    (jerk_stack) that do not involve the boundary velocity (rows 2..H of D1,
    rows 2..H-1 of D2), since these samples carry no boundary condition.
    """
    H = z.shape[1]
    v = sigma * z
    a = v @ problem.D1_matrix(H)[1:].T / dt
    j = v @ problem.D2_matrix(H)[1:].T / dt ** 2
    bad = (np.abs(v) > v_max).any(axis=1) | (np.abs(a) > a_max).any(axis=1) \
        | (np.abs(j) > j_max).any(axis=1)
    return float(bad.mean())


def sigma_eff_baseline(H: int, dt: float, n: int = 200_000, seed: int = 0,
                       threshold: float = 0.003, tol: float = 1e-4, hi: float = 1.0) -> float:
    """Largest admissible sigma for unfiltered white-noise samples (bisection)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, H))
    lo = 0.0
    while hi - lo > tol:
        mid = 0.5 * (lo + hi)
        if violation_rate(z, mid, dt) < threshold:
            lo = mid
        else:
            hi = mid
    return lo


def qp_limits(v_max=1.0, a_max=2.0, j_max=4.0, q_free=1e6):
    """Bounds of the QP diagnostic: velocity, acceleration and jerk only (the passage
    lists no position bound, so position rows get a bound far outside any reach)."""
    from .problem import JointLimits
    return JointLimits(-q_free, q_free, -v_max, v_max, -a_max, a_max, -j_max, j_max)


def sigma_eff_qp(z: np.ndarray, sigma: float, dt: float, v0: float = 0.0, tol: float = 1e-6,
                 cap: int = 60000):
    """Spread of the projected samples (Sec. III-C, QP paragraph): project sigma * z
    (rows are samples, shape [n, H]) with the velocity, acceleration and jerk bounds and
    x_1 = v0, then take the empirical standard deviation of all projected velocities
    (every sample and step pooled). Returns (std, projected samples [n, H]).

    The projection is the headline ADMM run to max(r_p, r_d) <= tol, block weights
    (1, 2.5/H, 4, 20), alpha 1.6.
    """
    from . import admm
    H = z.shape[1]
    r = admm.admm_joint(sigma * z, H, dt, qp_limits(), 0.0, v0, alpha=1.6, iters=cap, tol=tol,
                        check_every=50, weights=(1.0, 2.5 / H, 4.0, 20.0))
    return float(r.x.std()), r.x
