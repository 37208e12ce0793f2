"""Seeded synthetic inputs for the PWF hot path.

This package draws the inputs that the FP64 oracle and the HIP path share:
sample phase objects, diffuser transmissions, analytic ellipsoid phantoms and
their projections, and Poisson photon noise.  It holds none of the method's
arithmetic (no propagation, no intensity model, no gradient): the noise-free
speckle that Poisson noise is applied to is computed by whichever side uses
the data and handed to :func:`poisson_intensity`.
"""

from .generators import (  # noqa: F401
    BASE_SEED,
    Geometry,
    config_geometry,
    diffuser,
    ellipsoid_phantom,
    instance_inputs,
    phase_object,
    poisson_intensity,
    project_ellipsoids,
    roi_batch_specs,
    tomo_projection_inputs,
)
from .device_phantom import project_ellipsoids_device  # noqa: F401
