"""Brute force on small graphs: enumeration of states, the Hamiltonian as an explicit
sparse matrix, exact diagonalisation, exact variational energy and its gradient.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The matrix is built from the operator itself (Section 3 defines E_v as
<Psi|H|Psi>/<Psi|Psi>); it does not call the local-energy routine, so the two can
pin each other.  Spin-1/2 Heisenberg, ``H = sum_<ij> [Jz S^z_i S^z_j +
(Jxy/2)(S^+_i S^-_j + S^-_i S^+_j)]`` with ``S^z = s/2``.
"""
from __future__ import annotations

from itertools import combinations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def enumerate_sz0(n: int) -> np.ndarray:
    """All ``C(n, n/2)`` configurations with n/2 up spins, ``int8 [C, n]``."""
    if n % 2:
        raise ValueError("odd n has no S_z = 0 sector")
    states = []
    for ups in combinations(range(n), n // 2):
        s = -np.ones(n, dtype=np.int8)
        s[list(ups)] = 1
        states.append(s)
    return np.asarray(states, dtype=np.int8)


def enumerate_all(n: int) -> np.ndarray:
    """All ``2^n`` configurations (small n only)."""
    idx = np.arange(2 ** n)[:, None]
    bits = (idx >> np.arange(n)[None, :]) & 1
    return (2 * bits - 1).astype(np.int8)


def _keys(states: np.ndarray) -> np.ndarray:
    bits = (states > 0).astype(np.int64)
    return bits @ (np.int64(1) << np.arange(states.shape[1], dtype=np.int64))


def heisenberg_matrix(states: np.ndarray, edges, jz: float = 1.0, jxy: float = 1.0,
                      hb: float = 0.0, cb: float = 0.0):
    """Sparse H restricted to the span of ``states`` (closed under bond swaps); with
    ``hb, cb`` each bond also carries ``hb (S^z_i + S^z_j)/2 + cb``."""
    e = np.asarray(edges, dtype=np.int64)
    keys = _keys(states)
    index = {int(k): a for a, k in enumerate(keys)}
    rows, cols, vals = [], [], []
    for a, s in enumerate(states):
        diag = 0.0
        for i, j in e:
            diag += jz * (s[i] / 2.0) * (s[j] / 2.0) + hb * (s[i] / 2.0 + s[j] / 2.0) / 2.0 + cb
            if s[i] != s[j]:
                # S^+_i S^-_j + S^-_i S^+_j maps the pair to its swapped pair with amplitude 1
                t = s.copy()
                t[i], t[j] = s[j], s[i]
                rows.append(index[int(_keys(t[None, :])[0])])
                cols.append(a)
                vals.append(0.5 * jxy)
        rows.append(a)
        cols.append(a)
        vals.append(diag)
    dim = len(states)
    return sp.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def lowest_eigenpairs(Hm, k: int = 1):
    """Lowest ``k`` eigenvalues/vectors (dense ``eigh`` up to dim 4000, else Lanczos)."""
    dim = Hm.shape[0]
    if dim <= 4000:
        w, v = np.linalg.eigh(Hm.toarray())
        return w[:k], v[:, :k]
    w, v = spla.eigsh(Hm, k=k, which="SA", tol=1e-12)
    order = np.argsort(w)
    return w[order], v[:, order]


def variational_energy(psi, Hm) -> float:
    """``<psi|H|psi> / <psi|psi>`` (real for Hermitian H)."""
    psi = np.asarray(psi)
    num = np.vdot(psi, Hm @ psi)
    return float(num.real / np.vdot(psi, psi).real)


def psi_from_logpsi(lp) -> np.ndarray:
    """Complex amplitudes from ``[C, 2]`` (log|psi|, phase), max-shifted."""
    lp = np.asarray(lp, dtype=np.float64)
    a = lp[:, 0] - lp[:, 0].max()
    return np.exp(a) * np.exp(1j * lp[:, 1])


def exact_energy_of(logpsi_fn, states, Hm) -> float:
    return variational_energy(psi_from_logpsi(logpsi_fn(states)), Hm)
