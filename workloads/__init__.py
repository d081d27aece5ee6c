"""Seeded synthetic inputs for the projection QP.

This package holds only random-number draws and array shapes: it contains none
of the projection's arithmetic, so both the FP64 oracle and the HIP library's
tests and benchmark can use it without sharing any solver code.
"""

from .configs import (  # noqa: F401
    Bounds,
    Request,
    UR5E_BIMANUAL_BOUNDS,
    config1,
    config2,
    config3,
    config4_requests,
    config5_controllers,
    controller_samples,
    sigma_eff_workload,
    make_request,
    sinusoid_base,
)
