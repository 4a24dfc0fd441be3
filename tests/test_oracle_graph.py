"""Pins for the graph builders and the normalised adjacency of Eq. (1)."""
import numpy as np
import pytest

import oracle
import workloads as w


def _edge_set(e):
    return {(int(min(a, b)), int(max(a, b))) for a, b in e}


@pytest.mark.parametrize("L1,L2", [(2, 2), (3, 4), (6, 6), (12, 12)])
def test_kagome_counts_and_degrees(L1, L2):
    n, e = w.kagome(L1, L2)
    assert n == 3 * L1 * L2 and len(e) == 2 * n
    assert np.all(np.bincount(e.ravel(), minlength=n) == 4)


@pytest.mark.parametrize("L1,L2", [(3, 4), (4, 4), (12, 12)])
def test_triangular_counts_and_degrees(L1, L2):
    n, e = w.triangular(L1, L2)
    assert n == L1 * L2 and len(e) == 3 * n
    assert np.all(np.bincount(e.ravel(), minlength=n) == 6)


def test_kagome_translations_are_automorphisms():
    L = 4
    n, e = w.kagome(L, L)
    es = _edge_set(e)
    for dx, dy in [(1, 0), (0, 1), (3, 2)]:
        perm = np.empty(n, int)
        for y in range(L):
            for x in range(L):
                for s in range(3):
                    perm[3 * (x + L * y) + s] = 3 * ((x + dx) % L + L * ((y + dy) % L)) + s
        assert _edge_set(perm[e]) == es


def test_kagome_triangles():
    # every bond of a Kagome lattice lies in exactly one triangle (corner-sharing)
    n, e = w.kagome(3, 3)
    es = _edge_set(e)
    adj = [set() for _ in range(n)]
    for a, b in es:
        adj[a].add(b)
        adj[b].add(a)
    for a, b in es:
        assert len(adj[a] & adj[b]) == 1


def test_er_graph_connected_and_seeded():
    n, e1 = w.erdos_renyi_connected(100, 0.06, 0)
    _, e2 = w.erdos_renyi_connected(100, 0.06, 0)
    assert np.array_equal(e1, e2)
    assert w.lattices._connected(n, e1)
    deg = np.bincount(e1.ravel(), minlength=n)
    assert deg.min() >= 1 and deg.max() > deg.min()


@pytest.mark.parametrize("builder", [lambda: w.kagome(3, 3), lambda: w.triangular(3, 4),
                                     lambda: w.erdos_renyi_connected(30, 0.15, 3)])
def test_normalized_adjacency_spectrum(builder):
    # D^-1/2 A D^-1/2 is symmetric, its spectrum lies in [-1, 1], and sqrt(d) is an
    # eigenvector of eigenvalue 1 on a connected graph.  Row-normalisation D^-1 A or
    # a wrong degree would break symmetry or the eigenvector.
    n, e = builder()
    Ah = oracle.normalized_adjacency(n, e)
    assert np.allclose(Ah, Ah.T, atol=0, rtol=0)
    d = np.bincount(e.ravel(), minlength=n).astype(float)
    v = np.sqrt(d)
    assert np.allclose(Ah @ v, v, atol=1e-13)
    ev = np.linalg.eigvalsh(Ah)
    assert ev.max() == pytest.approx(1.0, abs=1e-12) and ev.min() >= -1 - 1e-12


def test_isolated_node_zero_row_and_bad_graphs():
    e = np.array([[0, 1], [1, 2]])
    Ah = oracle.normalized_adjacency(4, e)
    assert np.all(Ah[3] == 0) and np.all(Ah[:, 3] == 0)
    assert Ah[0, 1] == pytest.approx(1 / np.sqrt(2))
    with pytest.raises(ValueError):
        oracle.normalized_adjacency(3, np.array([[0, 0]]))
    with pytest.raises(ValueError):
        oracle.normalized_adjacency(3, np.array([[0, 1], [1, 0]]))
    with pytest.raises(ValueError):
        oracle.normalized_adjacency(3, np.array([[0, 3]]))
