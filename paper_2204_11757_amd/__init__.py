"""MI355X (gfx950) implementation of parallel spectrum-preserving graph
coarsening (Brissette, Huang, Slota, arXiv 2204.11757).

The computation lives in libspc.so (HIP kernels behind the C ABI declared in
include/spc.h); ``spc`` is its thin Python binding.
"""
from . import spc  # noqa: F401
from .spc import (  # noqa: F401
    DeviceGraph,
    Hierarchy,
    LevelStats,
    SpcError,
    coarsen_level,
    coarsen_to,
    lift,
    spectral_error,
    validate_graph,
)
