"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds workload *descriptions* only: grid sizes, spacings,
conductivities, time-step parameters and integer-indexed stimulus masks.  It
contains none of the method's arithmetic (no assembly, no ionic model, no time
stepping), so that both the FP64 oracle and the GPU library can consume the
same inputs without sharing any computational code.
"""
from .configs import CONFIGS, get_config, small_config  # noqa: F401
from .grids import box_mask, face_mask, grid_num_nodes  # noqa: F401
