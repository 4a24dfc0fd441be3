"""Flat FP64 parameter vector of the graph neural ansatz and its seeded initialisation.

Layout (an interface shared by every implementation; each one unpacks it itself):

    W_e[2][F]            embedding of the one-hot occupation (row 0: x=0 i.e. s=-1)
    b_e[F]
    W[nW][2F][F]         Eq. (1) weight; rows 0..F-1 multiply the neighbour message,
                         rows F..2F-1 multiply the node's own embedding
    b[nW][F]             Eq. (1) bias
    v_a[F+2], c_a        log-amplitude head on z = sum_i [H^L_i ; onehot(x_i)]
    v_p[F+2], c_p        phase head on the same z

with ``nW = 1`` when the layers share W and b (Section 2) and ``nW = L`` otherwise.
"""
from __future__ import annotations

import numpy as np


def theta_layout(F: int, L: int, tied: bool = True):
    """Ordered list of ``(name, shape, fan_in, fan_out)``; fans are ``None`` for biases."""
    nW = 1 if tied else L
    return [
        ("W_e", (2, F), 2, F),
        ("b_e", (F,), None, None),
        ("W", (nW, 2 * F, F), 2 * F, F),
        ("b", (nW, F), None, None),
        ("v_a", (F + 2,), F + 2, 1),
        ("c_a", (1,), None, None),
        ("v_p", (F + 2,), F + 2, 1),
        ("c_p", (1,), None, None),
    ]


def num_params(F: int, L: int, tied: bool = True) -> int:
    return int(sum(int(np.prod(shape)) for _, shape, _, _ in theta_layout(F, L, tied)))


def param_slices(F: int, L: int, tied: bool = True) -> dict:
    """``{name: (start, stop)}`` of each parameter block in the flat vector."""
    out, o = {}, 0
    for name, shape, _, _ in theta_layout(F, L, tied):
        size = int(np.prod(shape))
        out[name] = (o, o + size)
        o += size
    return out


def glorot_theta(F: int, L: int, tied: bool = True, seed: int = 0,
                 weight_scale: float = 1.0, bias_std: float = 0.0, real_head: bool = False) -> np.ndarray:
    """Glorot-normal weights ``N(0, 2/(fan_in+fan_out))`` drawn in layout order from
    ``PCG64(seed)``; biases are zero unless ``bias_std > 0`` (then drawn too, so that
    tests exercise every parameter).  ``weight_scale`` multiplies every weight.
    ``real_head`` zeroes the phase head after the draw: a positive wavefunction, the
    single real head the paper uses for hard-core bosons (Section 4).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for _, shape, fi, fo in theta_layout(F, L, tied):
        size = int(np.prod(shape))
        if fi is None:
            parts.append(rng.normal(0.0, bias_std, size) if bias_std > 0 else np.zeros(size))
        else:
            parts.append(weight_scale * rng.normal(0.0, np.sqrt(2.0 / (fi + fo)), size))
    theta = np.concatenate(parts).astype(np.float64)
    if real_head:
        sl = param_slices(F, L, tied)
        for name in ("v_p", "c_p"):
            theta[sl[name][0]:sl[name][1]] = 0.0
    return theta
