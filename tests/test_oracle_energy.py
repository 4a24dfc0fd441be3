"""Pins for the local energy (Section 3's E_x) and the explicit Hamiltonian.

* the explicit sparse H reproduces closed-form spectra (complete graph: total-spin
  formula; two sites: singlet/triplet; four-site ring: -2J);
* an exact eigenvector used as a table ansatz gives a constant E_loc equal to its
  eigenvalue (pins the off-diagonal amplitude and the diagonal);
* <psi|H|psi>/<psi|psi> equals the |psi|^2-weighted mean of E_loc for the GCN;
* zero heads (constant psi) give E_loc = |E|/4 for every configuration.
"""
from math import comb

import numpy as np
import pytest

import oracle
import workloads as w
from oracle import exact


def _table_fn(states, lp):
    keys = exact._keys(states)
    idx = {int(k): a for a, k in enumerate(keys)}

    def fn(c):
        return lp[[idx[int(k)] for k in exact._keys(np.asarray(c))]]
    return fn


@pytest.mark.parametrize("n", [4, 6, 8, 10])
def test_complete_graph_spectrum(n):
    # H = (J/2)(S_tot^2 - 3N/4) on K_N: eigenvalue (S(S+1) - 3N/4)/2 with multiplicity
    # C(N, N/2-S) - C(N, N/2-S-1) in the S_z = 0 sector
    _, e = w.complete_graph(n)
    st = exact.enumerate_sz0(n)
    ev = np.linalg.eigvalsh(exact.heisenberg_matrix(st, e).toarray())
    want = []
    for S in range(n // 2 + 1):
        mult = comb(n, n // 2 - S) - (comb(n, n // 2 - S - 1) if n // 2 - S - 1 >= 0 else 0)
        want += [0.5 * (S * (S + 1) - 0.75 * n)] * mult
    assert np.allclose(np.sort(ev), np.sort(want), atol=1e-12)


def test_two_sites_and_four_ring():
    st2 = exact.enumerate_sz0(2)
    ev2 = np.linalg.eigvalsh(exact.heisenberg_matrix(st2, np.array([[0, 1]])).toarray())
    assert np.allclose(ev2, [-0.75, 0.25], atol=1e-15)
    _, e4 = w.ring(4)
    ev4 = np.linalg.eigvalsh(exact.heisenberg_matrix(exact.enumerate_sz0(4), e4).toarray())
    assert ev4.min() == pytest.approx(-2.0, abs=1e-13)


def test_anisotropic_couplings_scale_separately():
    n, e = w.kagome(2, 2)
    st = exact.enumerate_sz0(n)
    Hz = exact.heisenberg_matrix(st, e, 1.0, 0.0)
    Hxy = exact.heisenberg_matrix(st, e, 0.0, 1.0)
    H = exact.heisenberg_matrix(st, e, 0.7, -1.9)
    assert abs(H - (0.7 * Hz - 1.9 * Hxy)).max() < 1e-15
    assert abs(Hz - sp_diag(Hz)).max() == 0


def sp_diag(M):
    import scipy.sparse as sp
    return sp.diags(M.diagonal())


@pytest.mark.parametrize("graph", ["kagome", "triangular", "er"])
def test_eigenvector_table_ansatz_gives_constant_local_energy(graph):
    if graph == "kagome":
        n, e = w.kagome(2, 2)
    elif graph == "triangular":
        n, e = w.triangular(3, 4)
    else:
        n, e = w.erdos_renyi_connected(12, 0.5, 0)
    st = exact.enumerate_sz0(n)
    Hm = exact.heisenberg_matrix(st, e)
    vals, vecs = exact.lowest_eigenpairs(Hm, 1)
    v = vecs[:, 0]
    keep = np.abs(v) > 1e-8
    lp = np.stack([np.log(np.abs(v) + 1e-300), np.where(v < 0, np.pi, 0.0)], 1)
    El = oracle.local_energy_generic(_table_fn(st, lp), st[keep], e)
    assert np.max(np.abs(El - vals[0])) < 1e-7
    assert vals[0] < 0


@pytest.mark.parametrize("graph", ["kagome", "triangular", "er"])
def test_weighted_local_energy_equals_quadratic_form(graph):
    if graph == "kagome":
        n, e = w.kagome(2, 2)
    elif graph == "triangular":
        n, e = w.triangular(3, 4)
    else:
        n, e = w.erdos_renyi_connected(12, 0.5, 0)
    F, L = 5, 2
    th = w.glorot_theta(F, L, True, seed=3, weight_scale=2.0, bias_std=0.5)
    st = exact.enumerate_sz0(n)
    Hm = exact.heisenberg_matrix(st, e, 0.8, 1.3)
    lp = oracle.forward(th, st, n, e, F, L)
    psi = exact.psi_from_logpsi(lp)
    El = oracle.local_energy(th, st, n, e, F, L, jz=0.8, jxy=1.3)
    p = np.abs(psi) ** 2 / np.sum(np.abs(psi) ** 2)
    Ev = exact.variational_energy(psi, Hm)
    assert abs(np.sum(p * El.real) - Ev) < 1e-12 * max(1, abs(Ev))
    assert abs(np.sum(p * El.imag)) < 1e-12          # Hermitian H: <E_loc> is real
    assert np.max(np.abs(El.imag)) > 1e-3             # ... though single E_loc are complex
    E0 = exact.lowest_eigenpairs(exact.heisenberg_matrix(st, e), 1)[0][0]
    Evj = exact.variational_energy(psi, exact.heisenberg_matrix(st, e))
    assert E0 - 1e-12 <= Evj <= len(e) / 4 + 1e-12   # variational sandwich


def test_zero_heads_give_quarter_bond_count_everywhere():
    n, e = w.kagome(2, 2)
    F, L = 4, 2
    th = w.glorot_theta(F, L, True, seed=1)
    sz = F + 2
    P = oracle.num_params(F, L, True)
    th[P - 2 * (sz + 1):] = 0.0                       # v_a, c_a, v_p, c_p
    st = exact.enumerate_all(n)[::7]                  # every S_z sector
    El = oracle.local_energy(th, st, n, e, F, L)
    assert np.all(El == len(e) / 4)


def test_fully_polarised_state_is_diagonal_only():
    n, e = w.triangular(3, 4)
    F, L = 4, 1
    th = w.glorot_theta(F, L, True, seed=2, weight_scale=2.0)
    up = np.ones((1, n), np.int8)
    assert oracle.local_energy(th, up, n, e, F, L, jz=1.0, jxy=5.0)[0] == len(e) / 4
    assert oracle.n_evals(up, e) == 1


def test_eval_count():
    n, e = w.kagome(2, 2)
    s = w.random_sz0_spins(50, n, 0)
    anti = (s[:, e[:, 0]] != s[:, e[:, 1]]).sum()
    assert oracle.n_evals(s, e) == 50 + anti
