"""Seeded synthetic inputs for the projection QP.

This package holds only random-number draws and array shapes: it contains none
of the projection's arithmetic, so both the FP64 oracle and the HIP library's
tests and benchmark can use it without sharing any solver code.
"""

from .recipes import (  # noqa: F401
    Bounds,
    Request,
    UR5E_BIMANUAL_BOUNDS,
    white_batch,
    mpc_batch,
    long_horizon_batch,
    uneven_requests,
    serving_controllers,
    poisson_arrivals,
    controller_samples,
    sigma_eff_workload,
    make_request,
    sinusoid_base,
)
