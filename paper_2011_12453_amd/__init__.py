"""MI355X (gfx950) implementation of the graph-neural-ansatz VMC hot path.

The compute runs in ``libgna.so`` (hand-written HIP kernels behind a C ABI, see
``include/gna.h``); this package only marshals arguments to it, and ``vmc`` sequences
the calls of Section 3's sampling-iteration loop.
"""
from .binding import (GNA, GnaError, LogPsi, library_path, load_library, FP64, FP32, BF16,
                      PRECISIONS, STAT_FIELDS)

__all__ = ["GNA", "GnaError", "LogPsi", "library_path", "load_library", "FP64", "FP32", "BF16",
           "PRECISIONS", "STAT_FIELDS"]
