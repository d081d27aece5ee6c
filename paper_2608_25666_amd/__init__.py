"""MI355X-native projection of sampled joint-velocity trajectories (PRISM's QP).

The work happens in libprism_proj.so (HIP for gfx950, C ABI in
include/prism_proj.h); this package only marshals arguments. Importing it does
not load the library; the first call does, and fails loudly if it is missing.
"""

from ._lib import (  # noqa: F401
    PREC_BF16, PREC_FP16, PREC_FP32, PrismError, load,
)
from .projector import Batch, Projector, default_block_weights, factor_host, options  # noqa: F401
from .server import Server, now_ns  # noqa: F401
