"""Named workloads shaped like the paper's experiments (Section 4), all synthetic.

Each preset fixes the graph, the ansatz shape and the batch; spins and weights are
drawn from the stated seeds.  The names say what the workload is.
"""
from __future__ import annotations

from dataclasses import dataclass

from .lattices import kagome, triangular, erdos_renyi_connected


@dataclass(frozen=True)
class Preset:
    name: str
    graph: str            # "kagome:L1xL2", "triangular:L1xL2", "er:N:p:seed"
    n_features: int
    n_layers: int
    batch: int
    spin_seed: int
    theta_seed: int = 0

    def build_graph(self):
        kind, _, rest = self.graph.partition(":")
        if kind == "kagome":
            a, b = (int(v) for v in rest.split("x"))
            return kagome(a, b)
        if kind == "triangular":
            a, b = (int(v) for v in rest.split("x"))
            return triangular(a, b)
        if kind == "er":
            n, p, seed = rest.split(":")
            return erdos_renyi_connected(int(n), float(p), int(seed))
        raise ValueError(self.graph)


PRESETS = {
    # 2x2x3 Kagome torus, 12 sites, 24 bonds; L=2, F=16; 1024 samples.
    "kagome12_L2F16": Preset("kagome12_L2F16", "kagome:2x2", 16, 2, 1024, 1001),
    # 6x6x3 Kagome torus, 108 sites, 216 bonds; L=4, F=32; 4096 samples.
    "kagome108_L4F32": Preset("kagome108_L4F32", "kagome:6x6", 32, 4, 4096, 1002),
    # 12x12 triangular torus, 144 sites, 432 bonds; L=4, F=32; 8192 samples.
    "triangular144_L4F32": Preset("triangular144_L4F32", "triangular:12x12", 32, 4, 8192, 1003),
    # G(100, 0.06) random graph, redrawn until connected; L=4, F=32; 4096 samples.
    "er100_L4F32": Preset("er100_L4F32", "er:100:0.06:0", 32, 4, 4096, 1004),
    # 12x12x3 Kagome torus, 432 sites, 864 bonds; L=6, F=64; 2048 samples.
    "kagome432_L6F64": Preset("kagome432_L6F64", "kagome:12x12", 64, 6, 2048, 1005),
}


def preset(name: str) -> Preset:
    return PRESETS[name]
