"""Seeded synthetic workloads shaped like the paper's bimanual MPC.

The paper plans for two 6-joint arms (12 joints, Sec. III-D 'Joint-wise
separability') and projects Gaussian samples around a mean velocity sequence
(Alg. 1, sampling step). Its MuJoCo/MJX task scenes are not available, so these
generators stand in for the projection's inputs:

* bounds |q| <= 2*pi rad, |v| <= 3.14 rad/s, |a| <= 8 rad/s^2, |j| <= 60 rad/s^3,
  identical for every joint;
* per request and joint: q0 ~ U(-pi, pi), v0 ~ U(-1.5, 1.5);
* samples either i.i.d. N(0, sigma^2) per step ("white"), or a smooth base
  trajectory (sum of three sinusoids of amplitude 1/3 rad/s each, frequencies
  U(0.2, 2.0) Hz, phases U(0, 2*pi), shared by all samples of a joint) plus
  i.i.d. N(0, 0.5^2) noise ("smooth").

Every array is drawn from ``numpy.random.Generator(PCG64(seed))`` in a fixed
order (q0, v0, base parameters, noise), so a (recipe, seed) pair names one input.
Samples use the library's layout: float32 ``[N][H][n_joints]`` row-major.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Bounds:
    """Per-joint lower/upper limits on position, velocity, acceleration, jerk."""

    q_min: np.ndarray
    q_max: np.ndarray
    v_min: np.ndarray
    v_max: np.ndarray
    a_min: np.ndarray
    a_max: np.ndarray
    j_min: np.ndarray
    j_max: np.ndarray

    @staticmethod
    def symmetric(nj: int, q: float, v: float, a: float, j: float) -> "Bounds":
        one = np.ones(nj, dtype=np.float64)
        return Bounds(-q * one, q * one, -v * one, v * one, -a * one, a * one, -j * one, j * one)

    def as_list(self):
        return [self.q_min, self.q_max, self.v_min, self.v_max,
                self.a_min, self.a_max, self.j_min, self.j_max]

    def subset(self, joints) -> "Bounds":
        return Bounds(*[np.asarray(b)[joints] for b in self.as_list()])


def UR5E_BIMANUAL_BOUNDS(nj: int) -> Bounds:
    """The workloads' limits: |q|<=2pi, |v|<=3.14, |a|<=8, |j|<=60 for every joint."""
    return Bounds.symmetric(nj, TWO_PI, 3.14, 8.0, 60.0)


@dataclasses.dataclass
class Request:
    """One projection call: samples of shape [N][H][nj] plus boundary values."""

    H: int
    nj: int
    dt: float
    bounds: Bounds
    q0: np.ndarray            # [nj] float64
    v0: np.ndarray            # [nj] float64
    samples: np.ndarray       # [N][H][nj] float32
    rho: float = 1.0
    iters: int = 100
    name: str = ""

    @property
    def N(self) -> int:
        return int(self.samples.shape[0])


def sinusoid_base(rng: np.random.Generator, H: int, nj: int, dt: float,
                  t0_steps: int = 0, freqs=None, phases=None):
    """Smooth base trajectory [H][nj]: sum of three sinusoids of amplitude 1/3.

    Step k (1-based) is evaluated at time (t0_steps + k) * dt, so a base for a
    later MPC step is the same curve shifted by whole steps.
    Returns (base, freqs, phases) so callers can re-evaluate a shifted base.
    """
    if freqs is None:
        freqs = rng.uniform(0.2, 2.0, size=(nj, 3))
    if phases is None:
        phases = rng.uniform(0.0, TWO_PI, size=(nj, 3))
    t = (t0_steps + np.arange(1, H + 1, dtype=np.float64)) * dt      # [H]
    arg = TWO_PI * freqs[None, :, :] * t[:, None, None] + phases[None, :, :]
    base = np.sin(arg).sum(axis=2) / 3.0                             # [H][nj]
    return base, freqs, phases


def make_request(seed: int, N: int, H: int, nj: int, dt: float, kind: str,
                 sigma: float = 1.0, noise: float = 0.5, rho: float = 1.0,
                 iters: int = 100, name: str = "") -> Request:
    """Draw one request. kind is 'white' (N(0, sigma^2)) or 'smooth' (base + N(0, noise^2))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    q0 = rng.uniform(-math.pi, math.pi, size=nj)
    v0 = rng.uniform(-1.5, 1.5, size=nj)
    if kind == "white":
        samples = rng.normal(0.0, sigma, size=(N, H, nj))
    elif kind == "smooth":
        base, _, _ = sinusoid_base(rng, H, nj, dt)
        samples = base[None, :, :] + rng.normal(0.0, noise, size=(N, H, nj))
    else:
        raise ValueError(f"unknown sample kind {kind!r}")
    return Request(H=H, nj=nj, dt=dt, bounds=UR5E_BIMANUAL_BOUNDS(nj), q0=q0, v0=v0,
                   samples=np.ascontiguousarray(samples, dtype=np.float32), rho=rho,
                   iters=iters, name=name)


def white_batch(seed: int = 0) -> Request:
    """12 joints, N=64, H=20, dt=0.05, white N(0,1) samples, rho=1, 200 iterations."""
    return make_request(seed, N=64, H=20, nj=12, dt=0.05, kind="white", sigma=1.0,
                        iters=200, name="white_N64_H20_J12_dt0.05")


def mpc_batch(seed: int = 0, N: int = 2048) -> Request:
    """12 joints, N=2048, H=50, dt=0.02, smooth base + N(0,0.5^2), rho=1, 100 iterations."""
    return make_request(seed, N=N, H=50, nj=12, dt=0.02, kind="smooth",
                        iters=100, name=f"mpc_N{N}_H50_J12_dt0.02")


def long_horizon_batch(seed: int = 0, N: int = 8192) -> Request:
    """12 joints, N=8192, H=100, dt=0.02, smooth generator, 100 iterations (90 reduced + 10 FP32)."""
    return make_request(seed, N=N, H=100, nj=12, dt=0.02, kind="smooth",
                        iters=100, name=f"long_N{N}_H100_J12_dt0.02")


def uneven_requests(seed: int = 0, n_requests: int = 64, n_choices=(128, 512, 2048, 4096),
                     h_choices=(20, 50, 100), nj_choices=(6, 12), dt_choices=(0.02, 0.05),
                     iters: int = 100) -> List[Request]:
    """Uneven batch: each request draws H, N, joint count and dt uniformly, then its own inputs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shapes = [(int(rng.choice(h_choices)), int(rng.choice(n_choices)),
               int(rng.choice(nj_choices)), float(rng.choice(dt_choices)))
              for _ in range(n_requests)]
    reqs = []
    for r, (H, N, nj, dt) in enumerate(shapes):
        reqs.append(make_request(seed * 1000 + r + 1, N=N, H=H, nj=nj, dt=dt, kind="smooth",
                                 iters=iters, name=f"uneven_r{r}_N{N}_H{H}_J{nj}_dt{dt}"))
    return reqs


@dataclasses.dataclass
class Controller:
    """A simulated MPC controller for the serving workload."""

    cid: int
    H: int
    N: int
    nj: int
    dt: float
    arrivals: np.ndarray        # request arrival times in seconds, ascending
    seed: int
    freqs: np.ndarray
    phases: np.ndarray
    q0: np.ndarray
    v0: np.ndarray


def serving_controllers(seed: int = 0, n_controllers: int = 32, rate_hz: float = 20.0,
                        duration_s: float = 60.0, n_choices=(128, 512, 2048, 4096),
                        h_choices=(20, 50, 100), nj_choices=(6, 12),
                        dt_choices=(0.02, 0.05)) -> List[Controller]:
    """Controllers with sizes drawn once each and Poisson arrivals at ``rate_hz``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ctrls = []
    for c in range(n_controllers):
        H = int(rng.choice(h_choices))
        N = int(rng.choice(n_choices))
        nj = int(rng.choice(nj_choices))
        dt = float(rng.choice(dt_choices))
        gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * duration_s * 2) + 16)
        t = np.cumsum(gaps)
        t = t[t < duration_s]
        freqs = rng.uniform(0.2, 2.0, size=(nj, 3))
        phases = rng.uniform(0.0, TWO_PI, size=(nj, 3))
        q0 = rng.uniform(-math.pi, math.pi, size=nj)
        v0 = rng.uniform(-1.5, 1.5, size=nj)
        ctrls.append(Controller(cid=c, H=H, N=N, nj=nj, dt=dt, arrivals=t,
                                seed=seed * 100000 + c * 1000 + 7, freqs=freqs, phases=phases,
                                q0=q0, v0=v0))
    return ctrls


def poisson_arrivals(n_controllers: int, rate_hz: float, duration_s: float,
                     seed: int = 1) -> List[np.ndarray]:
    """Poisson arrival times (seconds, ascending, < duration_s) for each of
    n_controllers at rate_hz: exponential gaps from their own generator, so the same
    controllers can be driven at several rates."""
    rng = np.random.Generator(np.random.PCG64(seed * 7 + int(round(rate_hz * 1000))))
    out = []
    for _ in range(n_controllers):
        gaps = rng.exponential(1.0 / rate_hz, size=int(rate_hz * duration_s * 2) + 16)
        t = np.cumsum(gaps)
        out.append(t[t < duration_s])
    return out


def controller_samples(ctrl: Controller, step: int, noise: float = 0.5,
                       N: Optional[int] = None) -> np.ndarray:
    """Samples for a controller's request number ``step``: base shifted by ``step`` steps + noise."""
    rng = np.random.Generator(np.random.PCG64(ctrl.seed + 7919 * (step + 1)))
    base, _, _ = sinusoid_base(rng, ctrl.H, ctrl.nj, ctrl.dt, t0_steps=step,
                               freqs=ctrl.freqs, phases=ctrl.phases)
    n = ctrl.N if N is None else N
    s = base[None, :, :] + rng.normal(0.0, noise, size=(n, ctrl.H, ctrl.nj))
    return np.ascontiguousarray(s, dtype=np.float32)


def sigma_eff_workload(n: int = 200_000, H: int = 15, seed: int = 0):
    """Single-joint diagnostic of Sec. III-C: n standard-normal velocity sequences of
    length H (scaled by the sampling sigma by the caller), bounds |v| <= 1, |a| <= 2,
    |j| <= 4 and no position bound (a limit of 1e6 rad stands in for none).
    Returns (z [n][H] float64, Bounds for one joint)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((n, H))
    b = Bounds.symmetric(1, 1e6, 1.0, 2.0, 4.0)
    return z, b
