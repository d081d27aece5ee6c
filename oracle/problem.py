"""The projection QP's constraint data, written out from the paper's definitions.

Test infrastructure only (see ``oracle/__init__``).

Paper references (Sec. III-D "Custom QP Solver"):
* velocity bounds, eq. (vel_bounds): the decision variable itself;
* position bounds, eqs. (pos_stack), (pos_bounds): forward-Euler positions
  theta_k = theta_init + dt * sum_{i<=k} thetadot_i, via the lower-triangular
  cumulative-sum matrix L;
* acceleration bounds, eqs. (acc_stack), (b_acc), (acc_bounds): first backward
  difference D1 / dt with thetadot_0 := thetadot_init entering through b_acc;
* jerk bounds, eqs. (jerk_stack), (D2_def), (b_jerk), (jerk_bounds): second
  difference D2 / dt^2 for k = 2..H, thetadot_0 := thetadot_init entering
  through b_jerk;
* compact QP, eqs. (compact_qp), (G_h_def), (A_b_def): G has (8H-2)*N_dof rows,
  A = [I 0 ... 0], b = thetadot_init.

Per-joint separability (Sec. III-D "Joint-wise separability") lets every
function here work on one joint; ``stacked_G_h`` builds the full Kronecker form
for the dimension checks.

Velocity-unit rows. The headline solver multiplies each row block of
G x <= h by a positive constant (1 for velocity, 1/dt for position, dt for
acceleration, dt^2 for jerk). Scaling an inequality by a positive number does
not change the feasible set, so the projection is unchanged; after scaling the
row matrix is the unit-free C = [I; L; D1; D2] with 4H-1 rows.
"""

from __future__ import annotations

import dataclasses

import numpy as np


# ---------------------------------------------------------------------------
# The paper's operator matrices
# ---------------------------------------------------------------------------

def L_matrix(H: int) -> np.ndarray:
    """Lower-triangular cumulative-sum matrix L (H x H) of eq. (pos_stack)."""
    return np.tril(np.ones((H, H)))


def D1_matrix(H: int) -> np.ndarray:
    """First-difference matrix D1 (H x H) of the acceleration paragraph: 1 on the
    diagonal, -1 on the first sub-diagonal."""
    return np.eye(H) - np.eye(H, k=-1)


def D2_matrix(H: int) -> np.ndarray:
    """Second-difference matrix D2 ((H-1) x H) of eq. (D2_def).

    Row r (0-based) holds the jerk at step k = r + 2 (1-based): its entries are
    1 at column r - 1 (absent for r = 0, where thetadot_init enters through
    b_jerk instead), -2 at column r and 1 at column r + 1.
    """
    D = np.zeros((H - 1, H))
    for r in range(H - 1):
        if r >= 1:
            D[r, r - 1] = 1.0
        D[r, r] = -2.0
        D[r, r + 1] = 1.0
    return D


def b_acc(H: int, dt: float, v0: float) -> np.ndarray:
    """Acceleration offset of eq. (b_acc) for one joint: (-v0/dt, 0, ..., 0)."""
    b = np.zeros(H)
    b[0] = -v0 / dt
    return b


def b_jerk(H: int, dt: float, v0: float) -> np.ndarray:
    """Jerk offset of eq. (b_jerk) for one joint: (v0/dt^2, 0, ..., 0), length H-1."""
    b = np.zeros(H - 1)
    b[0] = v0 / dt ** 2
    return b


# ---------------------------------------------------------------------------
# One joint: physical rows (paper scaling) and velocity-unit rows
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class JointLimits:
    """Scalar limits of one joint (position, velocity, acceleration, jerk)."""

    q_min: float
    q_max: float
    v_min: float
    v_max: float
    a_min: float
    a_max: float
    j_min: float
    j_max: float


def joint_limits(bounds, j: int) -> JointLimits:
    """Pick joint j's limits out of a ``workloads.Bounds``."""
    return JointLimits(*[float(np.asarray(b)[j]) for b in bounds.as_list()])


@dataclasses.dataclass
class JointRows:
    """Constraint rows lo <= C x <= hi for one joint (4H-1 rows, 4 blocks)."""

    C: np.ndarray      # (4H-1, H)
    lo: np.ndarray     # (4H-1,)
    hi: np.ndarray     # (4H-1,)
    H: int

    @property
    def blocks(self):
        """Row slices of the velocity, position, acceleration and jerk blocks."""
        H = self.H
        return (slice(0, H), slice(H, 2 * H), slice(2 * H, 3 * H), slice(3 * H, 4 * H - 1))


def physical_rows(H: int, dt: float, lim: JointLimits, q0: float, v0: float) -> JointRows:
    """Rows in physical units, eqs. (vel_bounds), (pos_bounds), (acc_bounds), (jerk_bounds).

    Each two-sided bound  lo_r <= C_r x + c_r <= hi_r  of the paper is stored as
    lo_r - c_r <= C_r x <= hi_r - c_r, with C_r = I, dt*L, D1/dt, D2/dt^2 and the
    affine parts c_r = 0, q0, b_acc, b_jerk.
    """
    C = np.vstack([np.eye(H), dt * L_matrix(H), D1_matrix(H) / dt, D2_matrix(H) / dt ** 2])
    c = np.concatenate([np.zeros(H), np.full(H, q0), b_acc(H, dt, v0), b_jerk(H, dt, v0)])
    lo = np.concatenate([np.full(H, lim.v_min), np.full(H, lim.q_min),
                         np.full(H, lim.a_min), np.full(H - 1, lim.j_min)]) - c
    hi = np.concatenate([np.full(H, lim.v_max), np.full(H, lim.q_max),
                         np.full(H, lim.a_max), np.full(H - 1, lim.j_max)]) - c
    return JointRows(C=C, lo=lo, hi=hi, H=H)


def row_scale(H: int, dt: float) -> np.ndarray:
    """Positive per-row factors that bring every block to velocity units (rad/s)."""
    return np.concatenate([np.ones(H), np.full(H, 1.0 / dt), np.full(H, dt),
                           np.full(H - 1, dt ** 2)])


def velocity_unit_rows(H: int, dt: float, lim: JointLimits, q0: float, v0: float) -> JointRows:
    """Physical rows multiplied by ``row_scale``: C becomes [I; L; D1; D2]."""
    p = physical_rows(H, dt, lim, q0, v0)
    s = row_scale(H, dt)
    return JointRows(C=s[:, None] * p.C, lo=s * p.lo, hi=s * p.hi, H=H)


# ---------------------------------------------------------------------------
# Full stacked form of the compact QP (all joints, Kronecker layout)
# ---------------------------------------------------------------------------

def stacked_G_h(H: int, dt: float, bounds, q0: np.ndarray, v0: np.ndarray):
    """G, h, A, b of eqs. (G_h_def) and (A_b_def) for N_dof joints.

    The stacked trajectory is step-major and joint-minor: entry k*N_dof + j is
    joint j at step k+1. Returns G ((8H-2)N_dof x H N_dof), h, A (N_dof x H N_dof), b.
    """
    nd = len(q0)
    I_nd = np.eye(nd)
    L = np.kron(L_matrix(H), I_nd)
    D1 = np.kron(D1_matrix(H), I_nd)
    D2 = np.kron(D2_matrix(H), I_nd)
    I_full = np.eye(H * nd)
    G = np.vstack([I_full, -I_full, dt * L, -dt * L, D1 / dt, -D1 / dt, D2 / dt ** 2, -D2 / dt ** 2])
    one_H = np.ones(H)
    one_H1 = np.ones(H - 1)
    qmin, qmax, vmin, vmax, amin, amax, jmin, jmax = [np.asarray(x, dtype=np.float64)
                                                      for x in bounds.as_list()]
    bacc = np.concatenate([-np.asarray(v0) / dt, np.zeros((H - 1) * nd)])
    bjerk = np.concatenate([np.asarray(v0) / dt ** 2, np.zeros((H - 2) * nd)])
    h = np.concatenate([
        np.kron(one_H, vmax), -np.kron(one_H, vmin),
        np.kron(one_H, qmax - q0), -np.kron(one_H, qmin - q0),
        np.kron(one_H, amax) - bacc, -np.kron(one_H, amin) + bacc,
        np.kron(one_H1, jmax) - bjerk, -np.kron(one_H1, jmin) + bjerk,
    ])
    A = np.hstack([np.eye(nd), np.zeros((nd, (H - 1) * nd))])
    b = np.asarray(v0, dtype=np.float64).copy()
    return G, h, A, b


def per_joint_G_h(H: int, dt: float, lim: JointLimits, q0: float, v0: float):
    """One joint's G = [C; -C] and h = [hi; -lo] in the paper's physical scaling."""
    p = physical_rows(H, dt, lim, q0, v0)
    return np.vstack([p.C, -p.C]), np.concatenate([p.hi, -p.lo])


def boundary_feasible(H: int, dt: float, lim: JointLimits, q0: float, v0: float) -> bool:
    """Necessary conditions for a nonempty feasible set given x_1 = v0.

    With x_1 = v0 the first velocity, position and acceleration rows are fixed
    numbers (v0, q0 + dt*v0 and zero acceleration), and the first jerk row
    (x_2 - v0)/dt^2 can only be met for every later choice if zero jerk is
    allowed. These conditions are necessary, not sufficient: a far-reaching
    horizon can still be infeasible, which the solver reports through a
    non-vanishing primal residual.
    """
    q1 = q0 + dt * v0
    return (lim.v_min <= v0 <= lim.v_max and lim.q_min <= q1 <= lim.q_max
            and lim.a_min <= 0.0 <= lim.a_max and lim.j_min <= 0.0 <= lim.j_max)
