"""Physical-unit constraint violations of velocity trajectories.

Test infrastructure only (see ``oracle/__init__``).

Sec. III-D, "From Joint-Velocity Sequences to Derivative Bounds": positions by
forward-Euler integration from theta_init (eq. (pos_stack)), accelerations by a
first backward difference with thetadot_0 := thetadot_init, jerks by
differencing consecutive accelerations for k = 2..H (eq. (jerk_stack)); plus
the boundary equality thetadot_1 = thetadot_init (eq. (A_b_def)).

This module computes those quantities by stepping through time in plain loops,
independently of the matrices in ``problem``, and reports the largest violation
of each bound in its own unit (rad, rad/s, rad/s^2, rad/s^3).
"""

from __future__ import annotations

import numpy as np


def violations(x: np.ndarray, dt: float, bounds, q0, v0):
    """Per (sample, joint) maxima of bound violations; x has layout [N][H][nj].

    Returns a dict of [N][nj] arrays: 'pos', 'vel', 'acc', 'jerk', 'eq'.
    """
    x = np.asarray(x, dtype=np.float64)
    N, H, nj = x.shape
    qmin, qmax, vmin, vmax, amin, amax, jmin, jmax = [np.asarray(b, dtype=np.float64)
                                                      for b in bounds.as_list()]
    out = {k: np.zeros((N, nj)) for k in ("pos", "vel", "acc", "jerk", "eq")}
    q = np.broadcast_to(np.asarray(q0, dtype=np.float64), (N, nj)).copy()
    prev_v = np.broadcast_to(np.asarray(v0, dtype=np.float64), (N, nj)).copy()
    prev_a = None
    for k in range(H):
        v = x[:, k, :]
        q = q + dt * v                               # theta_k = theta_{k-1} + dt * thetadot_k
        a = (v - prev_v) / dt                        # thetadot_0 = thetadot_init
        out["vel"] = np.maximum(out["vel"], np.maximum(v - vmax, vmin - v))
        out["pos"] = np.maximum(out["pos"], np.maximum(q - qmax, qmin - q))
        out["acc"] = np.maximum(out["acc"], np.maximum(a - amax, amin - a))
        if prev_a is not None:                       # jerk rows exist for k = 2..H
            jk = (a - prev_a) / dt
            out["jerk"] = np.maximum(out["jerk"], np.maximum(jk - jmax, jmin - jk))
        prev_v, prev_a = v, a
    out["eq"] = np.abs(x[:, 0, :] - np.asarray(v0, dtype=np.float64)[None, :])
    for k in out:
        out[k] = np.maximum(out[k], 0.0)
    return out


def max_violation(x, dt, bounds, q0, v0) -> dict:
    """Scalar maxima over all samples and joints, per block."""
    return {k: float(v.max()) if v.size else 0.0 for k, v in violations(x, dt, bounds, q0, v0).items()}
