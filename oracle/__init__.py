"""FP64 CPU oracle of preconditioned Wirtinger flow (test infrastructure).

Only the test-suite, the smoke entry point and the CPU-baseline leg of the
benchmark may import this package.  The product path (the HIP library and
its Python binding) never imports, links or calls it.
"""

from .pwf_oracle import *  # noqa: F401,F403
