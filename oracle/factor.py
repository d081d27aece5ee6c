"""The primal-update system of the ADMM iteration and its one-time factorization.

Test infrastructure only (see ``oracle/__init__``).

Sec. III-D, "Step 2: Primal update", eqs. (admm_primal) and (admm_KKT): the
primal step solves the saddle-point system

    M [x; mu] = [r; b],   M = [[I + delta G^T G, A^T], [A, 0]],

and "Pre-computable factorization" notes that M depends only on G, A and the
penalty, so one factorization serves every sample, joint and MPC step. For one
joint, A = e_1^T and b = v0 (eq. (A_b_def)).

The headline iteration uses the velocity-unit rows C (see ``problem``) with
penalty rho, so the (1,1) block is P = I + rho C^T C. ``KKTFactor`` factors M
once with an LU decomposition (scipy) and solves it for any number of
right-hand sides. ``reduced_inverse`` gives the equivalent closed form
x = K r + k v0 obtained by eliminating the multiplier mu:
Pi = P^{-1}, K = Pi - Pi e1 e1^T Pi / Pi_11, k = Pi e1 / Pi_11.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg


class KKTFactor:
    """LU factorization of M = [[P, e1], [e1^T, 0]] for one joint."""

    def __init__(self, P: np.ndarray):
        H = P.shape[0]
        M = np.zeros((H + 1, H + 1))
        M[:H, :H] = P
        M[:H, H] = 0.0
        M[0, H] = 1.0          # A^T = e1
        M[H, 0] = 1.0          # A = e1^T
        self.H = H
        self.M = M
        self.lu = scipy.linalg.lu_factor(M)

    def solve(self, r: np.ndarray, v0) -> np.ndarray:
        """Return x from M [x; mu] = [r; v0]; r has shape (H, ncols)."""
        r = np.atleast_2d(r.T).T if r.ndim == 1 else r
        ncols = r.shape[1]
        rhs = np.empty((self.H + 1, ncols))
        rhs[:self.H] = r
        rhs[self.H] = v0
        sol = scipy.linalg.lu_solve(self.lu, rhs)
        return sol[:self.H]

    def solve_with_multiplier(self, r: np.ndarray, v0):
        """Return (x, mu) of the saddle system."""
        ncols = r.shape[1]
        rhs = np.empty((self.H + 1, ncols))
        rhs[:self.H] = r
        rhs[self.H] = v0
        sol = scipy.linalg.lu_solve(self.lu, rhs)
        return sol[:self.H], sol[self.H]


def penalty_matrix(C: np.ndarray, rho: float) -> np.ndarray:
    """P = I + rho C^T C, the (1,1) block of M."""
    H = C.shape[1]
    return np.eye(H) + rho * (C.T @ C)


def reduced_inverse(P: np.ndarray):
    """(K, k) with x = K r + k v0 solving M [x; mu] = [r; v0] (Schur complement on mu)."""
    H = P.shape[0]
    Pi = np.linalg.inv(P)
    e1 = np.zeros(H)
    e1[0] = 1.0
    Pie1 = Pi @ e1
    K = Pi - np.outer(Pie1, Pie1) / Pie1[0]
    k = Pie1 / Pie1[0]
    return K, k
