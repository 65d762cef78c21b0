"""MI355X-native vielbein lattice Boltzmann step for binary fluids on a periodic torus.

The step itself runs in the HIP kernels of libtlb.so (C interface: include/tlb.h);
`binding.TorusGrid` marshals torch device buffers and streams into it, and `inputs` builds the
seeded synthetic initial conditions.
"""
from . import inputs  # noqa: F401
from .binding import (TorusGrid, TorusBatch, load_library, stable_dt, TlbError, FLAT,  # noqa: F401
                      CH_NO_ADVECTION, NO_GRAPH, WENO5, STRICT_DT, CH4)

__all__ = ["TorusGrid", "TorusBatch", "load_library", "stable_dt", "TlbError", "FLAT",
           "CH_NO_ADVECTION", "NO_GRAPH", "WENO5", "STRICT_DT", "CH4", "inputs"]
