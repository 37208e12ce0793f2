"""MI355X-native preconditioned Wirtinger flow (PWF) hot path.

The computation lives in ``libpwf.so`` (hand-written HIP for gfx950, C ABI in
``include/pwf.h``); this package marshals torch tensors into it.
"""

from .api import (  # noqa: F401
    DEFAULT_ALPHA,
    DEFAULT_ETA,
    DEFAULT_ETA_T,
    DEFAULT_GAMMA,
    DEFAULT_PRECOND_SCALE,
    PWF,
    Problem,
    background_quadratic,
    calibrate_source,
    diffuser_from_reference,
    fbp,
    fit_coherence,
    speckle_g2,
    problem_from_geometry,
    set_column_tile,
    set_graph_mode,
    set_merged_launch,
    set_row_plan,
    shell_correlation,
)
from ._lib import PwfError, load  # noqa: F401
from .autograd import PWFLoss, pwf_loss  # noqa: F401
