"""MI355X (gfx950) implementation of the graph-neural-ansatz VMC hot path.

The compute runs in ``libgna.so`` (hand-written HIP kernels behind a C ABI, see
``include/gna.h``); this package only marshals arguments to it, and ``vmc`` sequences
the calls of Section 3's sampling-iteration loop.

Typical use (device tensors; theta FP64 in the layout of ``include/gna.h``)::

    g = GNA(n_sites, edges, n_features=64, n_layers=6, precision="bf16_1x",
            eloc_mode="incremental", max_batch=2048)
    g.autotune(theta, spins)                      # optional: measure kernel shapes
    eloc, n_evals = g.local_energy(theta, spins)
    grad, stats, _ = g.isgo_grad(theta, spins, logpsi_old)
    g.sgd_update(theta, grad, lr)

Build with ``python -c "import __graft_entry__ as g; g.build()"`` (hipcc, gfx950).
"""
from .binding import (GNA, GnaError, LogPsi, library_path, load_library, FP64, FP32, BF16, BF16_1X,
                      PRECISIONS, STAT_FIELDS)

__all__ = ["GNA", "GnaError", "LogPsi", "library_path", "load_library", "FP64", "FP32", "BF16",
           "BF16_1X", "PRECISIONS", "STAT_FIELDS"]
