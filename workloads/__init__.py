"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package only *generates inputs*: triangulated PEC surfaces (the square
plate and the geodesic sphere of the paper's benchmark set, Section 2.1),
plane-wave incidence sets and seeded random test vectors. It contains none of
the method's arithmetic (no basis functions, Green's functions, projections or
integrals), so both the FP64 reference implementation and the GPU library can
consume its outputs without sharing any computation.
"""

from .meshes import (  # noqa: F401
    C0,
    Mesh,
    plate_mesh,
    sphere_mesh,
    sphere_subdivisions,
    wavelength,
)
from .waves import planewave_set, normal_incidence  # noqa: F401
from .vectors import random_current  # noqa: F401
from .configs import CONFIGS, config_mesh, config_meshes  # noqa: F401
