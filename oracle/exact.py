"""Exact solutions and optimality certificates for the projection QP.

Test infrastructure only (see ``oracle/__init__``).

These routines do not run ADMM; they pin what ADMM must converge to. The
projection of Sec. III-A, eq. (proj_cost) onto the polyhedron of
eqs. (proj_bounds)-(proj_boundary) is the unique minimiser of a strictly convex
quadratic, so:

* ``brute_force``: for tiny horizons, enumerate every set of active rows (at
  most H-1 of them, independent together with the equality x_1 = v0), project
  x~ onto the affine hull of that face, and keep the feasible candidate with
  the smallest objective. The true minimiser is the projection onto the affine
  hull of the face that contains it in its relative interior, and no feasible
  point is closer to x~, so the minimum over feasible candidates is x*.
* ``kkt_certificate``: x is the projection iff it is feasible and
  x - x~ + sum_i y_i C_i + mu e_1 = 0 with y_i >= 0 on rows at their upper
  bound and y_i <= 0 on rows at their lower bound (KKT conditions, sufficient
  for a convex QP). The multipliers are found with non-negative least squares
  (Lawson-Hanson, scipy.optimize.nnls); a zero residual certifies x.
* ``polish``: given an approximate solution and its multipliers, solve the
  equality-constrained least-squares problem on the identified active set and
  return the exact candidate (then certify it).
* ``slsqp``: scipy's SLSQP on the same problem, as a library cross-check.
"""

from __future__ import annotations

import itertools

import numpy as np
import scipy.optimize


def _eq_projection(xt, E, rhs):
    """argmin ||x - xt|| s.t. E x = rhs (E full row rank), for several rhs columns."""
    # x = xt - E^T lam,  E E^T lam = E xt - rhs
    EEt = E @ E.T
    lam = np.linalg.solve(EEt, (E @ xt)[:, None] - rhs)
    return xt[:, None] - E.T @ lam, lam


def brute_force(xt: np.ndarray, C: np.ndarray, lo: np.ndarray, hi: np.ndarray, v0: float,
                feas_tol: float = 1e-9):
    """Exact projection of one column by face enumeration (use for H <= 5)."""
    H = C.shape[1]
    m = C.shape[0]
    xt = np.asarray(xt, dtype=np.float64)
    e1 = np.zeros(H)
    e1[0] = 1.0
    best_x, best_f = None, np.inf
    for size in range(0, H):
        for S in itertools.combinations(range(m), size):
            E = np.vstack([e1[None, :], C[list(S)]]) if size else e1[None, :]
            if np.linalg.matrix_rank(E) < size + 1:
                continue
            # every lower/upper choice of the active rows
            choices = np.array(list(itertools.product((0, 1), repeat=size)), dtype=int) \
                if size else np.zeros((1, 0), dtype=int)
            rhs = np.empty((size + 1, len(choices)))
            rhs[0] = v0
            for t, i in enumerate(S):
                rhs[t + 1] = np.where(choices[:, t] == 0, lo[i], hi[i])
            X, _ = _eq_projection(xt, E, rhs)
            Cx = C @ X
            feas = np.all((Cx >= lo[:, None] - feas_tol) & (Cx <= hi[:, None] + feas_tol), axis=0)
            if not feas.any():
                continue
            f = 0.5 * np.sum((X - xt[:, None]) ** 2, axis=0)
            f[~feas] = np.inf
            k = int(np.argmin(f))
            if f[k] < best_f - 1e-15:
                best_f, best_x = f[k], X[:, k].copy()
    return best_x


def kkt_certificate(x: np.ndarray, xt: np.ndarray, C: np.ndarray, lo: np.ndarray,
                    hi: np.ndarray, v0: float, act_tol: float = 1e-7):
    """(max constraint violation, stationarity residual) for one column.

    Rows within ``act_tol`` of a bound may carry a multiplier of the sign that
    bound allows; the equality multiplier is free. Both numbers near zero
    certify that x is the projection.
    """
    x = np.asarray(x, dtype=np.float64)
    xt = np.asarray(xt, dtype=np.float64)
    H = C.shape[1]
    Cx = C @ x
    viol = max(0.0, float(np.max(Cx - hi)), float(np.max(lo - Cx)), abs(float(x[0] - v0)))
    up = np.where(Cx >= hi - act_tol)[0]
    dn = np.where(Cx <= lo + act_tol)[0]
    e1 = np.zeros(H)
    e1[0] = 1.0
    # x - xt + C_up^T a - C_dn^T b + (m1 - m2) e1 = 0, a, b, m1, m2 >= 0
    B = np.hstack([C[up].T, -C[dn].T, e1[:, None], -e1[:, None]])
    w, res = scipy.optimize.nnls(B, xt - x, maxiter=50 * B.shape[1] + 100)
    return viol, float(np.max(np.abs(B @ w - (xt - x))))


def polish(xt: np.ndarray, C: np.ndarray, lo: np.ndarray, hi: np.ndarray, v0: float,
           y: np.ndarray, y_tol: float = 1e-9):
    """Exact candidate from an approximate solution's multipliers y (constraint space).

    Rows with y_i > y_tol are taken active at hi, rows with y_i < -y_tol at lo.
    Dependent rows are dropped greedily so the active matrix has full row rank.
    """
    H = C.shape[1]
    e1 = np.zeros(H)
    e1[0] = 1.0
    rows = [e1]
    rhs = [v0]
    order = np.argsort(-np.abs(y))
    for i in order:
        if abs(y[i]) <= y_tol:
            break
        cand = np.vstack(rows + [C[i]])
        if np.linalg.matrix_rank(cand) < len(rows) + 1:
            continue
        rows.append(C[i])
        rhs.append(hi[i] if y[i] > 0 else lo[i])
    E = np.vstack(rows)
    X, _ = _eq_projection(np.asarray(xt, dtype=np.float64), E, np.array(rhs)[:, None])
    return X[:, 0]


def slsqp(xt: np.ndarray, C: np.ndarray, lo: np.ndarray, hi: np.ndarray, v0: float,
          x0=None, ftol: float = 1e-14):
    """scipy SLSQP solution of the same projection (cross-check, small H)."""
    xt = np.asarray(xt, dtype=np.float64)
    H = C.shape[1]
    if x0 is None:
        x0 = np.full(H, v0)
    cons = [
        {"type": "eq", "fun": lambda x: np.array([x[0] - v0]),
         "jac": lambda x: np.eye(1, H)},
        {"type": "ineq", "fun": lambda x: hi - C @ x, "jac": lambda x: -C},
        {"type": "ineq", "fun": lambda x: C @ x - lo, "jac": lambda x: C},
    ]
    r = scipy.optimize.minimize(lambda x: 0.5 * np.sum((x - xt) ** 2), x0,
                                jac=lambda x: x - xt, constraints=cons, method="SLSQP",
                                options={"ftol": ftol, "maxiter": 2000})
    return r.x
