"""Pins of the hard-core-boson model (Eq. 4) in the oracle: the occupation-basis
matrix built from the bosonic operators, its spin form, and closed forms."""
import numpy as np
import pytest

import oracle
from oracle import exact, hcb
import workloads as w


def _ring(n):
    return [(i, (i + 1) % n) for i in range(n)]


@pytest.mark.parametrize("t,V", [(1.0, 0.0), (0.3, 1.0), (1.0, 1.0), (0.0, 1.0)])
def test_spin_form_equals_boson_matrix(t, V):
    # n_i = (1 + s_i)/2 maps Eq. 4 onto the bond form with (jz, jxy, hb, cb)
    n, e = w.kagome(2, 2)
    occ = hcb.occupations(n, n // 2)
    Hb = hcb.hcb_matrix(occ, e, t, V).toarray()
    jz, jxy, hb_, cb = hcb.spin_couplings(t, V)
    states = (2 * occ.astype(np.int64) - 1).astype(np.int8)
    assert np.array_equal(states, exact.enumerate_sz0(n))          # same ordering
    Hs = exact.heisenberg_matrix(states, e, jz, jxy, hb_, cb).toarray()
    assert np.allclose(Hb, Hs, atol=1e-14)


@pytest.mark.parametrize("n", [6, 8, 10, 12])
def test_free_hard_core_bosons_on_a_ring(n):
    # V = 0: Jordan-Wigner gives free fermions, periodic for an odd number of particles
    # and antiperiodic for an even one; E0 = -2 t sum over the filled momenta cos k
    t, m = 1.0, n // 2
    Hb = hcb.hcb_matrix(hcb.occupations(n, m), _ring(n), t, 0.0)
    e0 = exact.lowest_eigenpairs(Hb, 1)[0][0]
    phi = 0.0 if m % 2 else 0.5
    ks = 2 * np.pi * (np.arange(n) + phi) / n
    eps = np.sort(-2 * t * np.cos(ks))
    assert abs(e0 - eps[:m].sum()) < 1e-10


def test_ground_state_is_positive_and_table_ansatz_is_exact():
    # hopping amplitudes are all -t < 0: the ground vector has one sign (Section 4), and
    # as a table ansatz it gives E_loc = E0 on every configuration, hb and cb included
    n, e = w.kagome(2, 2)
    t, V = 0.4, 1.0
    occ = hcb.occupations(n, n // 2)
    Hb = hcb.hcb_matrix(occ, e, t, V)
    e0, vec = exact.lowest_eigenpairs(Hb, 1)
    v = vec[:, 0] * np.sign(vec[0, 0])
    assert np.all(v > 0)
    states = (2 * occ.astype(np.int64) - 1).astype(np.int8)
    keys = {tuple(s): a for a, s in enumerate(states)}
    table = lambda c: np.stack([np.log(np.array([v[keys[tuple(x)]] for x in c])), np.zeros(len(c))], 1)
    jz, jxy, hb_, cb = hcb.spin_couplings(t, V)
    E = oracle.local_energy_generic(table, states, e, jz, jxy, hb=hb_, cb=cb)
    assert np.max(np.abs(E - e0[0])) < 1e-10


def test_classical_limit():
    # t = 0: the energy is V times the number of bonds joining two bosons; half filling on
    # a 2x2x3 Kagome torus cannot avoid occupied bonds, and the minimum is found by search
    n, e = w.kagome(2, 2)
    occ = hcb.occupations(n, n // 2)
    Hb = hcb.hcb_matrix(occ, e, 0.0, 1.0)
    direct = min(sum(int(o[i]) * int(o[j]) for i, j in e) for o in occ)
    assert abs(exact.lowest_eigenpairs(Hb, 1)[0][0] - direct) < 1e-12
    assert direct > 0


def test_real_head_gives_real_local_energy_and_zero_phase_gradient():
    # zero phase head: psi > 0, E_loc real, and the phase-head parameters get no gradient
    n, e = w.kagome(2, 2)
    F, L = 8, 2
    theta = w.glorot_theta(F, L, True, seed=2, weight_scale=1.5, bias_std=0.3, real_head=True)
    p = oracle.unpack_theta(theta, F, L)
    assert np.all(p["v_p"] == 0) and p["c_p"] == 0
    s = w.random_sz0_spins(16, n, 4)
    jz, jxy, hb_, cb = hcb.spin_couplings(0.5, 1.0)
    lp = oracle.logpsi(theta, s, n, e, F, L)
    g, stats, E = oracle.isgo_grad(theta, s, lp, n, e, F, L, jz=jz, jxy=jxy, hb=hb_, cb=cb)
    assert np.max(np.abs(E.imag)) == 0.0
    sl = w.param_slices(F, L, True)
    a, b = sl["v_p"]
    assert np.all(g[a:b] == 0) and g[sl["c_p"][0]] == 0
