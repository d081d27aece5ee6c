"""One iteration of the sampling optimizer around the projection (Alg. 1 without
the simulator): draw samples from N(nu, diag(sigma^2)), project them, score them
with a synthetic cost, weight them by a softmax of the cost (eq. (weight_update))
and update the mean and the diagonal covariance (eqs. (mean_update_new),
(cov_update_new)). The lowest-cost sample is returned as well (end of Alg. 1).

Test infrastructure only (see ``oracle/__init__``); plain NumPy, FP64 except where
a value is defined on 32-bit integers (the random-number generator).

Random numbers (the paper draws from the Gaussian; it names no generator): the
counter-based Philox4x32-10 generator (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), one call per sample element, turned
into a standard normal by the Box-Muller transform of its first two words
(23-bit uniforms).
The synthetic cost (the paper's costs come from MuJoCo rollouts, Sec. IV-C): a
joint-space tracking term w_pos * (theta_k - theta_ref_k)^2 on the positions
integrated from the projected velocities (eq. (pos_stack)) plus w_vel * v_k^2,
summed over steps and joints.
"""

from __future__ import annotations

import dataclasses

import numpy as np

from . import admm

M0, M1 = 0xD2511F53, 0xCD9E8D57           # Philox4x32 multipliers
W0, W1 = 0x9E3779B9, 0xBB67AE85           # Weyl key increments
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on arrays of counters.

    ctr: four uint32 arrays (or ints) c0..c3; key: two uint32 arrays k0, k1.
    Each round multiplies c0 and c2 by the two constants into 64-bit products,
    then the new counter is (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1,
    lo(M0*c0)); the key is bumped by the Weyl constants between rounds.
    """
    c = [np.asarray(v, dtype=np.uint64) & MASK for v in ctr]
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c[0] * np.uint64(M0)
        p1 = c[2] * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return [v.astype(np.uint32) for v in c]


def standard_normals(shape, seed: int, stream: int) -> np.ndarray:
    """Standard normals for every element e (row-major flat index) of `shape`.

    Element e takes Philox4x32-10 at counter (e mod 2^32, e div 2^32, stream mod
    2^32, stream div 2^32) with key (seed mod 2^32, seed div 2^32); its first two
    words w0, w1 give uniforms u = (floor(w / 2^9) + 1/2) / 2^23 in (0, 1) (23 bits,
    so u is exact in single precision as well), and z = sqrt(-2 ln u0) cos(2 pi u1).
    """
    n = int(np.prod(shape))
    e = np.arange(n, dtype=np.uint64)
    ctr = [e & MASK, e >> np.uint64(32), np.uint64(stream & MASK), np.uint64(stream >> 32)]
    key = [np.uint64(seed & MASK), np.uint64(seed >> 32)]
    w = philox4x32_10(ctr, key)
    u0 = ((w[0] >> np.uint32(9)).astype(np.float64) + 0.5) / 8388608.0
    u1 = ((w[1] >> np.uint32(9)).astype(np.float64) + 0.5) / 8388608.0
    z = np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)
    return z.reshape(shape)


def draw(nu: np.ndarray, sigma: np.ndarray, N: int, seed: int, stream: int) -> np.ndarray:
    """Samples x~ = nu + sigma * z, shape [N][H][nj] (nu, sigma: [H][nj])."""
    z = standard_normals((N,) + nu.shape, seed, stream)
    return nu[None] + sigma[None] * z


def tracking_cost(x: np.ndarray, q0, dt: float, theta_ref: np.ndarray, w_pos: float,
                  w_vel: float) -> np.ndarray:
    """c_n = sum_k sum_j w_pos (theta_kj - ref_kj)^2 + w_vel x_kj^2, with
    theta_k = q0 + dt sum_{i<=k} x_i (forward Euler, eq. (pos_stack)). x: [N][H][nj]."""
    theta = np.asarray(q0, dtype=np.float64)[None, None, :] + dt * np.cumsum(x, axis=1)
    return (w_pos * (theta - theta_ref[None]) ** 2 + w_vel * x ** 2).sum(axis=(1, 2))


def softmax_weights(c: np.ndarray, tau: float) -> np.ndarray:
    """omega_n = exp(-c_n / tau) / sum_m exp(-c_m / tau) (eq. (weight_update)),
    evaluated with the minimum cost subtracted first (the same ratio)."""
    a = np.exp(-(c - c.min()) / tau)
    return a / a.sum()


def moments(x: np.ndarray, omega: np.ndarray, eps: float):
    """nu' = sum_n omega_n x_n; Sigma' = diag(sum_n omega_n (x_n - nu')^2) + eps
    (eqs. (mean_update_new), (cov_update_new)). Returns (nu' [H][nj], var' [H][nj])."""
    nu = np.einsum("n,nhj->hj", omega, x)
    var = np.einsum("n,nhj->hj", omega, (x - nu[None]) ** 2) + eps
    return nu, var


@dataclasses.dataclass
class PlanResult:
    samples: np.ndarray     # [N][H][nj] drawn x~
    x: np.ndarray           # [N][H][nj] projected
    cost: np.ndarray        # [N]
    omega: np.ndarray       # [N]
    nu: np.ndarray          # [H][nj]
    var: np.ndarray         # [H][nj]
    best: int


def plan_step(nu, sigma, N, seed, stream, H, dt, bounds, q0, v0, theta_ref, w_pos, w_vel,
              tau, eps, iters, rho=1.0, alpha=1.0, weights=None, tol=None,
              check_every=10) -> PlanResult:
    """Sample, project (the headline ADMM), score, weight, update the moments."""
    xt = draw(np.asarray(nu, np.float64), np.asarray(sigma, np.float64), N, seed, stream)
    r = admm.solve_request(xt, H, dt, bounds, q0, v0, rho=rho, alpha=alpha, iters=iters,
                           tol=tol, check_every=check_every, weights=weights)
    c = tracking_cost(r.x, q0, dt, np.asarray(theta_ref, np.float64), w_pos, w_vel)
    om = softmax_weights(c, tau)
    m, v = moments(r.x, om, eps)
    return PlanResult(samples=xt, x=r.x, cost=c, omega=om, nu=m, var=v, best=int(np.argmin(c)))
