"""Seeded synthetic workloads for the sparse lattice-Boltzmann step.

This package only generates inputs: voxel label grids of synthetic vessels, the
iolet (inlet/outlet) descriptors that go with them, and seeded random
population deviations.  It holds none of the method's arithmetic (no lattice,
no equilibrium, no streaming); both the FP64 checker and the GPU path consume
the arrays it produces.

The patient 3D rotational-angiography geometries the paper measures on
(Section 4, Table 2) are not available; the generators here stand in for them
with the same structure: thin, sparse vessels, a single inlet with a pulsatile
velocity, pressure outlets.
"""

from .geometry import (  # noqa: F401
    SOLID,
    FLUID,
    Iolet,
    Geometry,
    pipe,
    aneurysm,
    tree,
    couette,
    channel,
    duct,
    closed_box,
    periodic_box,
    config_geometry,
)
from .states import random_deviations  # noqa: F401
