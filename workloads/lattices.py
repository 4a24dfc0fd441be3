"""Edge lists for the geometries of the paper's experiments (Section 4, Fig. 2 and 3).

Every builder returns an ``int32`` array of shape ``[n_edges, 2]`` with ``i < j`` in
each row, no self-loops and no repeated unordered pair.  Periodic boundaries are
built into the edge list itself, which is how the paper treats them (Section 2:
the boundary sites connect to the opposite side while constructing A).
"""
from __future__ import annotations

import numpy as np


def _canonical(pairs, n_sites: int) -> np.ndarray:
    out = []
    seen = set()
    for a, b in pairs:
        a, b = int(a), int(b)
        if a == b:
            raise ValueError(f"self-loop at site {a}")
        key = (min(a, b), max(a, b))
        if key in seen:
            raise ValueError(f"duplicate bond {key}; lattice too small for periodic wrap")
        seen.add(key)
        out.append(key)
    arr = np.asarray(out, dtype=np.int32).reshape(-1, 2)
    if arr.size and (arr.min() < 0 or arr.max() >= n_sites):
        raise ValueError("site index out of range")
    return arr


def kagome(l1: int, l2: int | None = None) -> tuple[int, np.ndarray]:
    """Kagome torus of ``l1 x l2`` unit cells, three sites per cell (Section 4, Fig. 3).

    Site ``3*(x + l1*y) + sigma`` with ``sigma`` in {A, B, C} = {0, 1, 2}.  Each cell
    carries an up-triangle A-B, A-C, B-C and the three bonds of a down-triangle
    A(x,y)-B(x-1,y), A(x,y)-C(x,y-1), B(x,y)-C(x+1,y-1), all indices mod the torus.
    Gives 2N bonds, every site of degree 4.  ``l1, l2 >= 2``.
    """
    l2 = l1 if l2 is None else l2
    if l1 < 2 or l2 < 2:
        raise ValueError("kagome torus needs at least 2x2 cells")
    n = 3 * l1 * l2

    def site(x, y, s):
        return 3 * ((x % l1) + l1 * (y % l2)) + s

    pairs = []
    for y in range(l2):
        for x in range(l1):
            a, b, c = site(x, y, 0), site(x, y, 1), site(x, y, 2)
            pairs += [(a, b), (a, c), (b, c)]
            pairs += [(a, site(x - 1, y, 1)), (a, site(x, y - 1, 2)), (b, site(x + 1, y - 1, 2))]
    return n, _canonical(pairs, n)


def triangular(l1: int, l2: int | None = None) -> tuple[int, np.ndarray]:
    """Triangular torus ``l1 x l2`` (Section 4, Fig. 2b).

    Site ``x + l1*y``, bonds to (x+1, y), (x, y+1), (x-1, y+1) mod the torus.
    Gives 3N bonds, every site of degree 6.  ``l1, l2 >= 3``.
    """
    l2 = l1 if l2 is None else l2
    if l1 < 3 or l2 < 3:
        raise ValueError("triangular torus needs at least 3x3 sites")
    n = l1 * l2

    def site(x, y):
        return (x % l1) + l1 * (y % l2)

    pairs = []
    for y in range(l2):
        for x in range(l1):
            s = site(x, y)
            pairs += [(s, site(x + 1, y)), (s, site(x, y + 1)), (s, site(x - 1, y + 1))]
    return n, _canonical(pairs, n)


def _connected(n: int, edges: np.ndarray) -> bool:
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    seen = np.zeros(n, bool)
    stack = [0]
    seen[0] = True
    while stack:
        u = stack.pop()
        for v in adj[u]:
            if not seen[v]:
                seen[v] = True
                stack.append(v)
    return bool(seen.all())


def erdos_renyi_connected(n: int, p: float, seed: int, max_tries: int = 10000) -> tuple[int, np.ndarray]:
    """Random graph: each pair present independently with probability ``p`` (Section 4).

    Pairs ``i < j`` are visited in row-major order and kept when a ``PCG64(seed)``
    uniform draw is below ``p``; the whole graph is redrawn from the same stream
    until it is connected.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    for _ in range(max_tries):
        keep = rng.random(iu.size) < p
        edges = np.stack([iu[keep], ju[keep]], axis=1).astype(np.int32)
        if edges.shape[0] and _connected(n, edges):
            return n, edges
    raise RuntimeError("no connected graph drawn")


def complete_graph(n: int) -> tuple[int, np.ndarray]:
    """All ``n(n-1)/2`` pairs; its Heisenberg spectrum has a closed form."""
    iu, ju = np.triu_indices(n, k=1)
    return n, np.stack([iu, ju], axis=1).astype(np.int32)


def ring(n: int) -> tuple[int, np.ndarray]:
    """Periodic chain of ``n >= 3`` sites."""
    return n, _canonical([(i, (i + 1) % n) for i in range(n)], n)
