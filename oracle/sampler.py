"""Metropolis spin-swap sampler, FP64 oracle (Section 3: states drawn with
probability proportional to |Psi|^2 by a Markov chain).

TEST INFRASTRUCTURE ONLY (see the package docstring).

One chain per batch row.  A sweep is N proposals.  Each proposal draws one
Philox4x32-10 block (counter = proposal index, chain), picks a bond uniformly;
an aligned bond is an identity step, an anti-aligned one proposes the swap
``s -> s^ij`` and accepts it when ``u < exp(2 Re[log psi(s^ij) - log psi(s)])``.
"""
from __future__ import annotations

import numpy as np

from .philox import philox_uniform_and_edge


def metropolis_sweeps(logpsi_fn, spins, logpsi, edges, n_sweeps: int, seed: int,
                      counter_base: int = 0):
    """Advance every chain by ``n_sweeps * N`` proposals.

    ``logpsi_fn(spins[b, N]) -> [b, 2]``; ``logpsi[B, 2]`` must be the chains'
    current values.  Returns new ``(spins, logpsi, n_accept[B])`` (inputs untouched).
    """
    s = np.array(spins, dtype=np.int8, copy=True)
    lp = np.array(logpsi, dtype=np.float64, copy=True)
    e = np.asarray(edges, dtype=np.int64)
    B, N = s.shape
    acc = np.zeros(B, dtype=np.int64)
    chains = np.arange(B, dtype=np.uint64)
    for t in range(n_sweeps * N):
        step = np.uint64(counter_base + t)
        k, u = philox_uniform_and_edge(np.full(B, step, dtype=np.uint64), chains, seed, len(e))
        i, j = e[k, 0], e[k, 1]
        rows = np.arange(B)
        anti = np.nonzero(s[rows, i] != s[rows, j])[0]
        if anti.size == 0:
            continue
        prop = s[anti].copy()
        ia, ja = i[anti], j[anti]
        r = np.arange(anti.size)
        prop[r, ia], prop[r, ja] = s[anti, ja], s[anti, ia]
        lp_new = logpsi_fn(prop)
        ok = u[anti] < np.exp(2.0 * (lp_new[:, 0] - lp[anti, 0]))
        take = anti[ok]
        s[take] = prop[ok]
        lp[take] = lp_new[ok]
        acc[take] += 1
    return s, lp, acc
