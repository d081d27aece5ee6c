"""ADMM iterations for the projection QP, in FP64.

Test infrastructure only (see ``oracle/__init__``).

The problem (Sec. III-A, eqs. (proj_cost)-(proj_boundary); Sec. III-D,
eq. (compact_qp)), per joint and column (one sample of one joint):

    x* = argmin_x 1/2 ||x - x~||^2   s.t.  x_1 = v0,  lo <= C x <= hi,

with C, lo, hi the velocity-unit rows of ``problem.velocity_unit_rows``.

Headline iteration ("admm"). The paper's splitting (Sec. III-D, "ADMM
Solver"): a slack projection (Step 1, eq. (admm_zeta)), a primal solve with the
pre-factored KKT matrix (Step 2, eqs. (admm_primal), (admm_KKT)), and a
residual-driven multiplier update (Step 3, eq. (admm_dual)). As printed, the
multiplier lives in the primal space and is absent from the slack step, which
makes every feasible point a fixed point; this module therefore keeps the same
three steps and the same factorization but carries the multiplier y in the
constraint space (the standard scaled ADMM). Its fixed point is the exact
projection. With relaxation alpha (1 = none) one iteration is

    x+  = solution of M [x; mu] = [x~ + rho C^T (z - y/rho); v0]      (Step 2)
    s^  = alpha C x+ + (1 - alpha) z
    z+  = clip(s^ + y/rho, lo, hi)                                    (Step 1)
    y+  = y + rho (s^ - z+)                                           (Step 3)

Initialization (the paper gives none). Within an iteration the paper takes
the slack step before the primal step (Step 1 uses the previous iterate x^l),
so the first pass here is a slack step and a multiplier step from the
starting point, with the previous slack taken as C x0:
    x0 = x~ with x0_1 := v0 (or a warm x_w with its first step set to v0),
    s0 = C x0,   z0 = clip(s0 + y_w/rho),   y0 = y_w + rho (s0 - z0),
where y_w is a warm multiplier (0 for a cold start). A feasible sample with
x~_1 = v0 gives z0 = s0 and y0 = 0 and is a fixed point from the start.
A warm start may also carry the previous slack z_w: the first pass then is an
ordinary relaxed step s^ = alpha s0 + (1 - alpha) z_w (z_w = s0 when absent).

Residuals (per column, velocity units, rad/s):
    r_p = max_i |(C x)_i - z_i|                         primal feasibility gap
    r_d = max_{k>=2} |x_k - x~_k + (C^T y)_k|           stationarity gap
The stationarity row k = 1 is excluded because the equality multiplier mu of
x_1 = v0 absorbs it.

Early exit. With a tolerance, each column stops at the first check point
(iteration 0, every ``check_every`` iterations, and its cap) where its own
max(r_p, r_d) <= tol. The paper gives no stopping rule (Sec. III-D
"Convergence" speaks only of low residuals), so the plain reading is per
column; how a solver groups columns for stopping is its own business and is
checked against this per-column definition, not built into it. ``iters`` may
also be an array with one count per column: column c then runs exactly
iters[c] iterations (or stops earlier at the tolerance).

Block penalties. The paper's penalty delta is one scalar. A positive diagonal
penalty R = rho * diag(w_V, w_Q, w_A, w_J) (one weight per constraint block)
keeps the same splitting, the same three steps and a single reusable
factorization (P = I + C^T R C); it only changes the metric of the augmented
term, so the fixed point is still the projection. With weights the steps read
    x+ : M [x; mu] = [x~ + C^T (R z - y); v0],   P = I + C^T R C
    z+ = clip(s^ + R^-1 y, lo, hi),   y+ = y + R (s^ - z+),
and the start is z0 = clip(s0 + R^-1 y_w), y0 = y_w + R (s0 - z0). Unit
weights give the scalar-penalty iteration above.

``literal_joint`` runs the iteration exactly as printed (paper scaling of G,
delta = rho, primal-space lambda, dual step delta/2) for comparison only.
"""

from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from . import problem
from .factor import KKTFactor, penalty_matrix



@dataclasses.dataclass
class JointResult:
    x: np.ndarray        # (ncols, H)
    r_p: np.ndarray      # (ncols,)
    r_d: np.ndarray      # (ncols,)
    iters: np.ndarray    # (ncols,) int
    z: np.ndarray        # (ncols, 4H-1)
    y: np.ndarray        # (ncols, 4H-1)


def residuals(C, x, xt, z, y):
    """(r_p, r_d) per column for states given as (rows, ncols) arrays."""
    r_p = np.max(np.abs(C @ x - z), axis=0)
    stat = x - xt + C.T @ y
    r_d = np.max(np.abs(stat[1:]), axis=0) if x.shape[0] > 1 else np.zeros(x.shape[1])
    return r_p, r_d


def block_penalty(H: int, rho: float, weights=None) -> np.ndarray:
    """Per-row penalty rho * w_b for the velocity, position, acceleration, jerk blocks."""
    w = (1.0, 1.0, 1.0, 1.0) if weights is None else tuple(float(v) for v in weights)
    return rho * np.concatenate([np.full(H, w[0]), np.full(H, w[1]), np.full(H, w[2]),
                                 np.full(H - 1, w[3])])


def start_state(xt: np.ndarray, C: np.ndarray, lo: np.ndarray, hi: np.ndarray,
                R: np.ndarray, v0: float, alpha: float, warm_x=None, warm_y=None,
                warm_z=None):
    """Starting point and the first slack/multiplier pass (reading R3).

    xt: (H, ncols) samples; lo, hi, R: (rows, 1). Returns (x0, z0, y0), all
    (rows or H, ncols): x0 = x~ (or the warm iterate) with x0_1 := v0, s0 = C x0,
    s^0 = alpha s0 + (1 - alpha) z_w (z_w = s0 when absent),
    z0 = clip(s^0 + R^-1 y_w), y0 = y_w + R (s^0 - z0).
    """
    ncols = xt.shape[1]
    x = (xt.copy() if warm_x is None else np.asarray(warm_x, dtype=np.float64).T.copy())
    x[0, :] = v0
    y = (np.zeros((C.shape[0], ncols)) if warm_y is None
         else np.asarray(warm_y, dtype=np.float64).T.copy())
    s0 = C @ x
    zw = s0 if warm_z is None else np.asarray(warm_z, dtype=np.float64).T
    shat0 = alpha * s0 + (1.0 - alpha) * zw
    z = np.clip(shat0 + y / R, lo, hi)
    y = y + R * (shat0 - z)
    return x, z, y


def relaxed_step(xt: np.ndarray, z: np.ndarray, y: np.ndarray, C: np.ndarray, lo: np.ndarray,
                 hi: np.ndarray, R: np.ndarray, fac: KKTFactor, v0: float, alpha: float):
    """One ADMM iteration on the paper's splitting, multiplier in constraint space.

    Step 2 (eqs. (admm_primal), (admm_KKT)): x+ solves
        M [x; mu] = [x~ + C^T (R z - y); v0],  P = I + C^T R C,
    i.e. x+ minimises 1/2||x - x~||^2 + 1/2||C x - z + R^-1 y||_R^2 with x_1 = v0.
    Relaxation: s^ = alpha C x+ + (1 - alpha) z (alpha = 1: none).
    Step 1 (eq. (admm_zeta), slack projection): z+ = clip(s^ + R^-1 y, lo, hi).
    Step 3 (eq. (admm_dual), multiplier step): y+ = y + R (s^ - z+).
    Arrays are (rows or H, ncols); lo, hi, R are (rows, 1). Returns (x+, z+, y+).
    """
    r = xt + C.T @ (R * z - y)
    x_new = fac.solve(r, v0)
    shat = alpha * (C @ x_new) + (1.0 - alpha) * z
    z_new = np.clip(shat + y / R, lo, hi)
    y_new = y + R * (shat - z_new)
    return x_new, z_new, y_new


def admm_joint(xt_cols: np.ndarray, H: int, dt: float, lim: problem.JointLimits,
               q0: float, v0: float, rho: float = 1.0, alpha: float = 1.0,
               iters=100, tol: Optional[float] = None, check_every: int = 10,
               warm_x: Optional[np.ndarray] = None,
               warm_y: Optional[np.ndarray] = None, weights=None,
               warm_z: Optional[np.ndarray] = None) -> JointResult:
    """Headline ADMM for the columns of one joint.

    xt_cols: (ncols, H) samples x~. ``iters``: one count for every column or an
    array of per-column counts. With ``tol`` None each column runs exactly its
    count; otherwise the count is its cap and the column stops at the first
    check point where its own max(r_p, r_d) <= tol.
    ``weights``: block penalty weights (w_V, w_Q, w_A, w_J), default all 1.
    """
    rows = problem.velocity_unit_rows(H, dt, lim, q0, v0)
    C, lo, hi = rows.C, rows.lo[:, None], rows.hi[:, None]
    R = block_penalty(H, rho, weights)[:, None]
    fac = KKTFactor(np.eye(H) + C.T @ (R * C))
    xt = np.asarray(xt_cols, dtype=np.float64).T.copy()         # (H, ncols)
    ncols = xt.shape[1]
    cap = np.broadcast_to(np.asarray(iters, dtype=np.int64), (ncols,)).copy()
    if np.any(cap < 0):
        raise ValueError("iteration counts must be >= 0")
    x, z, y = start_state(xt, C, lo, hi, R, v0, alpha, warm_x, warm_y, warm_z)

    done = np.zeros(ncols, dtype=bool)
    n_done = cap.copy()

    def check(l, cols):
        if tol is None:
            return
        r_p, r_d = residuals(C, x, xt, z, y)
        hit = cols & ~done & (np.maximum(r_p, r_d) <= tol)
        done[hit] = True
        n_done[hit] = l

    check(0, np.ones(ncols, dtype=bool))
    for l in range(1, int(cap.max(initial=0)) + 1):
        act = ~done & (l <= cap)
        if not act.any():
            break
        x[:, act], z[:, act], y[:, act] = relaxed_step(xt[:, act], z[:, act], y[:, act], C, lo,
                                                       hi, R, fac, v0, alpha)
        check(l, act & ((l % check_every == 0) | (l == cap)))
    r_p, r_d = residuals(C, x, xt, z, y)
    return JointResult(x=x.T.copy(), r_p=r_p, r_d=r_d, iters=n_done, z=z.T.copy(), y=y.T.copy())


@dataclasses.dataclass
class RequestResult:
    x: np.ndarray        # [N][H][nj] float64
    r_p: np.ndarray      # [N][nj]
    r_d: np.ndarray      # [N][nj]
    iters: np.ndarray    # [N][nj]
    y: np.ndarray        # [N][nj][4H-1]
    z: np.ndarray        # [N][nj][4H-1]


def solve_request(samples: np.ndarray, H: int, dt: float, bounds, q0, v0,
                  rho: float = 1.0, alpha: float = 1.0, iters=100,
                  tol: Optional[float] = None, check_every: int = 10,
                  warm_x: Optional[np.ndarray] = None,
                  warm_y: Optional[np.ndarray] = None, weights=None,
                  warm_z: Optional[np.ndarray] = None) -> RequestResult:
    """Project every sample of a request (layout [N][H][nj]), joint by joint.

    ``iters``: one count (or cap) for all columns, or an [N][nj] array of
    per-column counts."""
    samples = np.asarray(samples)
    N, H_, nj = samples.shape
    assert H_ == H
    iters = np.asarray(iters, dtype=np.int64)
    per_col = iters.ndim > 0
    if per_col:
        iters = np.broadcast_to(iters, (N, nj))
    x = np.zeros((N, H, nj))
    r_p = np.zeros((N, nj))
    r_d = np.zeros((N, nj))
    it = np.zeros((N, nj), dtype=np.int64)
    y = np.zeros((N, nj, 4 * H - 1))
    z = np.zeros((N, nj, 4 * H - 1))
    for j in range(nj):
        lim = problem.joint_limits(bounds, j)
        res = admm_joint(samples[:, :, j], H, dt, lim, float(q0[j]), float(v0[j]), rho=rho,
                         alpha=alpha, iters=iters[:, j] if per_col else int(iters), tol=tol,
                         check_every=check_every,
                         warm_x=None if warm_x is None else warm_x[:, :, j],
                         warm_y=None if warm_y is None else warm_y[:, j, :],
                         weights=weights,
                         warm_z=None if warm_z is None else warm_z[:, j, :])
        x[:, :, j] = res.x
        r_p[:, j] = res.r_p
        r_d[:, j] = res.r_d
        it[:, j] = res.iters
        y[:, j, :] = res.y
        z[:, j, :] = res.z
    return RequestResult(x=x, r_p=r_p, r_d=r_d, iters=it, y=y, z=z)


def shift_rows(a: np.ndarray, H: int) -> np.ndarray:
    """Advance every row block of a [N][nj][4H-1] array by one step, repeating the last."""
    out = np.empty_like(a)
    for sl in problem.JointRows(C=None, lo=None, hi=None, H=H).blocks:
        blk = a[:, :, sl]
        out[:, :, sl] = np.concatenate([blk[:, :, 1:], blk[:, :, -1:]], axis=2)
    return out


def shift_state(x: np.ndarray, y: np.ndarray, H: int):
    """Warm start for the next MPC step: advance x and every row block of y by one
    step, repeating the last entry of each block (x: [N][H][nj], y: [N][nj][4H-1])."""
    xs = np.concatenate([x[:, 1:, :], x[:, -1:, :]], axis=1)
    return xs, shift_rows(y, H)


def advance_warm_start(x: np.ndarray, y: np.ndarray, z: np.ndarray, H: int, v0_new):
    """Warm start of the next MPC step from a previous result (the paper does not
    define one; this is the library's reading, stated here in full).

    Time advances by dt, so step k of the new problem takes step k + 1 of the old
    one, the last step repeating, block by block for the rows:
    * the iterate: x'_k = x_{k+1}, x'_H = x_H, and x'_1 = v0_new;
    * the multiplier y and the slack's deviation from the constraint values,
      d = z - C x (zero at convergence), are advanced the same way;
    * the slack is rebuilt on the new iterate, z' = C x' + d'.
    The acceleration row of step 1 is fixed by x_1 = v0 and restarts with zero
    multiplier and zero deviation. C = [I; L; D1; D2] in velocity units; the
    boundary values sit in the row bounds, so they need no handling here.

    x: [N][H][nj]; y, z: [N][nj][4H-1]; v0_new: [nj]. Returns (x', y', z').
    """
    C = np.vstack([np.eye(H), problem.L_matrix(H), problem.D1_matrix(H), problem.D2_matrix(H)])
    A0 = 2 * H                                   # row: acceleration of step 1
    x = np.asarray(x, dtype=np.float64)
    xs = np.concatenate([x[:, 1:, :], x[:, -1:, :]], axis=1)
    xs[:, 0, :] = np.asarray(v0_new, dtype=np.float64)[None, :]
    d = np.asarray(z, dtype=np.float64) - np.einsum("rh,nhj->njr", C, x)
    ys = shift_rows(np.asarray(y, dtype=np.float64), H)
    ds = shift_rows(d, H)
    ys[:, :, A0] = 0.0
    ds[:, :, A0] = 0.0
    zs = np.einsum("rh,nhj->njr", C, xs) + ds
    return xs, ys, zs


# ---------------------------------------------------------------------------
# The iteration exactly as printed in the paper (comparison flag)
# ---------------------------------------------------------------------------

def literal_joint(xt_cols: np.ndarray, H: int, dt: float, lim: problem.JointLimits,
                  q0: float, v0: float, delta: float = 1.0, iters: int = 100,
                  x_init: Optional[np.ndarray] = None, lam_init: Optional[np.ndarray] = None,
                  return_lam: bool = False):
    """Sec. III-D, eqs. (admm_zeta), (admm_primal)/(admm_KKT), (admm_dual), verbatim.

    G, h in the paper's physical scaling (eq. (G_h_def), one joint), penalty delta,
    lambda in the primal space, lambda_0 = 0 and x_0 = x~ with x_1 := v0 unless
    ``lam_init`` / ``x_init`` are given. Returns (x (ncols, H), max constraint
    violation per column), and lambda (ncols, H) as a third item with ``return_lam``.
    """
    G, h = problem.per_joint_G_h(H, dt, lim, q0, v0)
    fac = KKTFactor(np.eye(H) + delta * (G.T @ G))
    xt = np.asarray(xt_cols, dtype=np.float64).T.copy()
    x = xt.copy() if x_init is None else np.asarray(x_init, dtype=np.float64).T.copy()
    x[0, :] = v0
    lam = np.zeros_like(xt) if lam_init is None else np.asarray(lam_init, dtype=np.float64).T.copy()
    hh = h[:, None]
    for _ in range(iters):
        zeta = np.maximum(0.0, hh - G @ x)                                  # Step 1
        x = fac.solve(delta * (G.T @ (hh - zeta)) + lam + xt, v0)           # Step 2
        lam = lam - 0.5 * delta * (G.T @ (G @ x - hh + zeta))               # Step 3
    viol = np.maximum(0.0, np.max(G @ x - hh, axis=0))
    if return_lam:
        return x.T.copy(), viol, lam.T.copy()
    return x.T.copy(), viol
