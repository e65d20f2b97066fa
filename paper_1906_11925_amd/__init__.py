"""MI355X-native sparse lattice-Boltzmann time step (HemeLB's method, arXiv 1906.11925).

The hot path lives in ``libhemelb_lb.so`` (HIP kernels for gfx950 behind the C
ABI of ``include/hemelb_lb.h``); this package holds its ctypes binding and
build script.  Importing it does not touch the GPU.
"""

from .lb import LB, links, plan, plan_geometry, copy_probe, relaxation_time  # noqa: F401
from .lib import HemelbError, load  # noqa: F401
