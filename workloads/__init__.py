"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This package builds graphs (edge lists), flat parameter vectors and spin batches.
It holds none of the method's arithmetic: no adjacency normalisation, no forward
pass, no energy.  Both the CPU oracle and the HIP path receive exactly these
arrays as inputs.
"""
from .lattices import kagome, triangular, erdos_renyi_connected, complete_graph, ring
from .params import theta_layout, num_params, glorot_theta, param_slices
from .spins import random_sz0_spins, random_spins
from .presets import PRESETS, preset

__all__ = [
    "kagome", "triangular", "erdos_renyi_connected", "complete_graph", "ring",
    "theta_layout", "num_params", "glorot_theta", "param_slices",
    "random_sz0_spins", "random_spins", "PRESETS", "preset",
]
