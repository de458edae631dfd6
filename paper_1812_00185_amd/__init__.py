"""MI355X-native coarse-grid incremental pressure-projection (CGP) library.

The compute path is the HIP library libcgp.so (C-ABI in include/cgp.h);
``CGP`` is its thin Python front end.  There is no CPU fallback: if the
library is not built, loading it raises.
"""
from ._native import load as load_library  # noqa: F401
from .solver import CGP, StepState  # noqa: F401
