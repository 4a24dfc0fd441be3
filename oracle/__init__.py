"""FP64 CPU oracle for the graph-neural-ansatz VMC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this package:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.  It
shares no code with the HIP library and is written from the paper's definitions
(Eq. 1-3, Sections 2-3) in plain NumPy/SciPy, without blocking or fusion.
"""
from .philox import philox4x32_10, philox_uniform_and_edge
from .gna import (
    unpack_theta, num_params, normalized_adjacency, forward, logpsi,
    local_energy, local_energy_generic, n_evals, isgo_stats, logpsi_vjp, isgo_grad,
    sgd_update,
)
from .sampler import metropolis_sweeps
from . import exact
from . import hcb
from .group import group_duplicates

__all__ = [
    "philox4x32_10", "philox_uniform_and_edge", "unpack_theta", "num_params",
    "normalized_adjacency", "forward", "logpsi", "local_energy", "local_energy_generic",
    "n_evals", "isgo_stats", "logpsi_vjp", "isgo_grad", "sgd_update",
    "metropolis_sweeps", "exact", "hcb", "group_duplicates",
]
