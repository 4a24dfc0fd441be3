"""Grouping of duplicated sampled states into unique states with counts (Section 3,
the sampler's output before it is sharded to the workers).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The definition: the unique rows of the batch, each once, in the order of their first
occurrence, with the number of times each occurs.  Written as a plain dictionary pass
over the rows; no hashing beyond Python's own exact byte keys.
"""
import numpy as np


def group_duplicates(spins):
    """``(unique[U, N] int8, counts[U] float64, index[B])`` with
    ``unique[index[b]] == spins[b]`` for every row ``b``."""
    s = np.asarray(spins, dtype=np.int8)
    first = {}
    order = []
    counts = []
    index = np.empty(s.shape[0], dtype=np.int64)
    for b in range(s.shape[0]):
        key = s[b].tobytes()
        g = first.get(key)
        if g is None:
            g = len(order)
            first[key] = g
            order.append(b)
            counts.append(0)
        counts[g] += 1
        index[b] = g
    uniq = s[order] if order else s[:0]
    return uniq, np.asarray(counts, dtype=np.float64), index
