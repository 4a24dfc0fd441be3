"""Pins for the oracle's forward pass (Eq. 1 and the readout of Section 2).

The paper prints no values, so the pins are closed forms of special cases,
symmetries, and agreement between independent formulations of the aggregation.
"""
import numpy as np
import pytest

import oracle
import workloads as w
from oracle import exact

F, L = 6, 3


def _theta(F=F, L=L, tied=True, seed=0):
    return w.glorot_theta(F, L, tied, seed=seed, weight_scale=1.3, bias_std=0.4)


def _set(theta, F, L, tied, **blocks):
    p = oracle.unpack_theta(theta.copy(), F, L, tied)
    t = theta.copy()
    o = 0
    for name, shape, _, _ in w.theta_layout(F, L, tied):
        size = int(np.prod(shape))
        if name in blocks:
            t[o:o + size] = np.broadcast_to(blocks[name], shape).ravel()
        o += size
    return t


@pytest.mark.parametrize("tied", [True, False])
def test_three_aggregation_formulations_agree(tied):
    n, e = w.erdos_renyi_connected(20, 0.2, 1)
    th = _theta(tied=tied)
    s = w.random_spins(16, n, 5)
    a = oracle.forward(th, s, n, e, F, L, tied, "dense")
    b = oracle.forward(th, s, n, e, F, L, tied, "sparse")
    c = oracle.forward(th, s, n, e, F, L, tied, "edges")
    assert np.max(np.abs(a - b)) < 1e-12 and np.max(np.abs(a - c)) < 1e-12


def test_no_layers_depends_only_on_counts():
    # L = 0: z = (sum_i tanh(W_e[x_i] + b_e), n0, n1) only counts the spins
    n, e = w.kagome(2, 2)
    th = _theta(L=0)
    st = exact.enumerate_sz0(n)
    lp = oracle.forward(th, st, n, e, F, 0)
    assert np.ptp(lp[:, 0]) < 1e-12 and np.ptp(lp[:, 1]) < 1e-12


def test_zero_layer_weights_closed_form():
    # W = 0 in Eq. (1): every node's embedding becomes tanh(b) after the first layer,
    # so z = (N tanh(b), n_down, n_up) whatever the graph
    n, e = w.triangular(3, 4)
    th = _set(_theta(), F, L, True, W=0.0)
    p = oracle.unpack_theta(th, F, L, True)
    s = w.random_spins(8, n, 2)
    lp = oracle.forward(th, s, n, e, F, L)
    nup = (s > 0).sum(1)
    z = np.concatenate([np.repeat(n * np.tanh(p["b"][0])[None], 8, 0),
                        np.stack([n - nup, nup], 1)], 1)
    assert np.allclose(lp[:, 0], z @ p["v_a"] + p["c_a"], atol=1e-12, rtol=0)
    assert np.allclose(lp[:, 1], z @ p["v_p"] + p["c_p"], atol=1e-12, rtol=0)


def test_message_weight_zero_makes_graph_irrelevant():
    # rows 0..F-1 of W multiply the neighbour message; zero them and the ansatz no
    # longer sees the edges (a swapped concatenation order would fail this)
    th = _theta()
    p = oracle.unpack_theta(th, F, L, True)
    W = p["W"].copy()
    W[:, :F, :] = 0
    th0 = _set(th, F, L, True, W=W)
    n1, e1 = w.kagome(2, 2)
    _, e2 = w.erdos_renyi_connected(12, 0.5, 7)
    s = w.random_sz0_spins(10, n1, 3)
    assert np.allclose(oracle.forward(th0, s, n1, e1, F, L), oracle.forward(th0, s, n1, e2, F, L),
                       atol=1e-13, rtol=0)
    # ... and with the full W it does
    assert not np.allclose(oracle.forward(th, s, n1, e1, F, L), oracle.forward(th, s, n1, e2, F, L))


def test_self_weight_zero_on_edgeless_graph_closed_form():
    # rows F..2F-1 multiply the node's own embedding; zero them on a graph without
    # edges and every layer output is tanh(b)
    th = _theta()
    p = oracle.unpack_theta(th, F, L, True)
    W = p["W"].copy()
    W[:, F:, :] = 0
    th0 = _set(th, F, L, True, W=W)
    n = 10
    s = w.random_spins(4, n, 9)
    _, act = oracle.forward(th0, s, n, np.zeros((0, 2), int), F, L, keep=True)
    assert np.allclose(act["H"][-1], np.tanh(p["b"][0]), atol=1e-15, rtol=0)


def test_zero_heads_constant():
    th = _set(_theta(), F, L, True, v_a=0.0, v_p=0.0, c_a=0.7, c_p=-0.2)
    n, e = w.kagome(2, 2)
    lp = oracle.forward(th, w.random_spins(7, n, 1), n, e, F, L)
    assert np.all(lp[:, 0] == 0.7) and np.all(lp[:, 1] == -0.2)


def test_tied_equals_untied_with_repeated_weights():
    th_t = _theta(tied=True)
    p = oracle.unpack_theta(th_t, F, L, True)
    th_u = _set(w.glorot_theta(F, L, False, 0), F, L, False,
                W_e=p["W_e"], b_e=p["b_e"], W=np.repeat(p["W"], L, 0), b=np.repeat(p["b"], L, 0),
                v_a=p["v_a"], c_a=p["c_a"], v_p=p["v_p"], c_p=p["c_p"])
    n, e = w.triangular(3, 3)
    s = w.random_spins(5, n, 4)
    assert np.array_equal(oracle.forward(th_t, s, n, e, F, L, True), oracle.forward(th_u, s, n, e, F, L, False))


@pytest.mark.parametrize("kind", ["kagome", "triangular"])
def test_torus_translation_invariance(kind):
    th = _theta()
    if kind == "kagome":
        Lc = 4
        n, e = w.kagome(Lc, Lc)
        perm = np.array([3 * (((c // 3) % Lc + 1) % Lc + Lc * ((c // 3) // Lc)) + c % 3 for c in range(n)])
    else:
        Lc = 4
        n, e = w.triangular(Lc, Lc)
        perm = np.array([((c % Lc) + 1) % Lc + Lc * (c // Lc) for c in range(n)])
    s = w.random_sz0_spins(6, n, 8)
    t = np.empty_like(s)
    t[:, perm] = s                          # spin at site c moves to site perm[c]
    a = oracle.forward(th, s, n, e, F, L)
    b = oracle.forward(th, t, n, e, F, L)
    assert np.max(np.abs(a - b)) < 1e-12


def test_relabelling_equivariance():
    th = _theta(tied=False)
    n, e = w.erdos_renyi_connected(16, 0.3, 11)
    rng = np.random.default_rng(0)
    perm = rng.permutation(n)
    e2 = perm[e]
    s = w.random_spins(6, n, 12)
    s2 = np.empty_like(s)
    s2[:, perm] = s
    a = oracle.forward(th, s, n, e, F, L, False)
    b = oracle.forward(th, s2, n, e2, F, L, False)
    assert np.max(np.abs(a - b)) < 1e-12
