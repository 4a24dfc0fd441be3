"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Written from the published definition: a 4x32-bit counter and a 2x32-bit key;
each of 10 rounds multiplies counter words 0 and 2 by two fixed odd constants,
keeps the 64-bit products' high and low halves, and recombines them with XOR
against counter words 1, 3 and the key; the key is advanced by two Weyl
constants between rounds.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.

    ``ctr``: uint32-compatible array ``[..., 4]``; ``key``: ``[..., 2]`` (broadcast).
    Returns uint32 ``[..., 4]``.
    """
    c = np.asarray(ctr, dtype=np.uint64) & _MASK
    k = np.asarray(key, dtype=np.uint64) & _MASK
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = np.broadcast_to(k[..., 0], c0.shape), np.broadcast_to(k[..., 1], c0.shape)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0            # < 2^64, exact in uint64
        p1 = _M1 * c2
        hi0, lo0 = p0 >> _S32, p0 & _MASK
        hi1, lo1 = p1 >> _S32, p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def philox_uniform_and_edge(step, chain, seed, n_edges):
    """Draws for one Metropolis proposal.

    Counter = (low32(step), high32(step), chain, 0), key = (low32(seed), high32(seed)).
    Word 0 picks the bond ``(w0 * n_edges) >> 32``; word 1 gives the uniform
    ``u = (w1 + 0.5) * 2^-32`` in (0, 1).
    """
    step = np.asarray(step, dtype=np.uint64)
    chain = np.asarray(chain, dtype=np.uint64)
    step, chain = np.broadcast_arrays(step, chain)
    ctr = np.stack([step & _MASK, step >> _S32, chain & _MASK, np.zeros_like(step)], axis=-1)
    s = np.uint64(seed)
    out = philox4x32_10(ctr, np.array([s & _MASK, s >> _S32], dtype=np.uint64))
    w0 = out[..., 0].astype(np.uint64)
    w1 = out[..., 1].astype(np.float64)
    edge = ((w0 * np.uint64(n_edges)) >> _S32).astype(np.int64)
    u = (w1 + 0.5) * 2.0 ** -32
    return edge, u
