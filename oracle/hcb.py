"""Hard-core bosons of Eq. 4: ``H = -t sum_<ij> (b+_i b_j + b+_j b_i) + V sum_<ij> n_i n_j``.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The matrix is built in the occupation basis from the bosonic operators themselves
(two bosons never share a site; hopping moves one boson along a bond), independently
of the spin form used by the local energy.  With ``n_i = (1 + s_i)/2`` the model is a
bond Hamiltonian of the form ``oracle.gna.local_energy_generic`` takes:

    V n_i n_j = V/4 (1 + s_i + s_j + s_i s_j)        -> jz = V, hb = V, cb = V/4
    -t (b+_i b_j + h.c.) = -t [n_i != n_j] (swap)    -> jxy = -2 t

(parity unpinned by the paper, which prints no energies; pinned by the independent
matrix below and by closed forms in the tests).
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp


def spin_couplings(t: float, V: float):
    """``(jz, jxy, hb, cb)`` of the bond Hamiltonian equal to Eq. 4."""
    return float(V), float(-2.0 * t), float(V), float(V) / 4.0


def occupations(n: int, n_bosons: int) -> np.ndarray:
    """All occupations with ``n_bosons`` bosons on ``n`` sites, ``int8 [C, n]`` in {0, 1}."""
    out = []
    for occ in combinations(range(n), n_bosons):
        v = np.zeros(n, dtype=np.int8)
        v[list(occ)] = 1
        out.append(v)
    return np.asarray(out, dtype=np.int8)


def hcb_matrix(occ: np.ndarray, edges, t: float, V: float):
    """Sparse Eq. 4 on the span of the occupations ``occ`` (fixed boson number).

    ``b+_i b_j`` acting on a state with ``n_j = 1, n_i = 0`` gives the state with the
    boson moved from j to i, amplitude 1 (hard-core bosons: no signs); otherwise 0.
    """
    e = np.asarray(edges, dtype=np.int64)
    keys = {tuple(int(x) for x in v): a for a, v in enumerate(occ)}
    rows, cols, vals = [], [], []
    for a, v in enumerate(occ):
        diag = 0.0
        for i, j in e:
            diag += V * float(v[i]) * float(v[j])
            for src, dst in ((j, i), (i, j)):       # b+_dst b_src
                if v[src] == 1 and v[dst] == 0:
                    w = v.copy()
                    w[src], w[dst] = 0, 1
                    rows.append(keys[tuple(int(x) for x in w)])
                    cols.append(a)
                    vals.append(-t)
        rows.append(a)
        cols.append(a)
        vals.append(diag)
    dim = len(occ)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))
