"""Pins for the Philox4x32-10 stream and the Metropolis spin-swap sampler."""
import os

import numpy as np
import pytest
from scipy import stats as sst

import oracle
import workloads as w
from oracle import exact
from oracle.philox import philox4x32_10, philox_uniform_and_edge

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(np.array(v[:4], np.uint64), np.array(v[4:6], np.uint64))
        assert [int(x) for x in out] == v[6:]


def test_draws_uniform():
    k, u = philox_uniform_and_edge(np.arange(200000, dtype=np.uint64), 3, 12345, 24)
    assert k.min() == 0 and k.max() == 23
    assert sst.chisquare(np.bincount(k, minlength=24)).pvalue > 1e-4
    assert 0 < u.min() and u.max() < 1
    assert sst.kstest(u, "uniform").pvalue > 1e-4


def _setup(F=4, L=2, seed=5):
    n, e = w.kagome(2, 2)
    th = w.glorot_theta(F, L, True, seed=seed, weight_scale=2.5, bias_std=0.5)
    st = exact.enumerate_sz0(n)
    lp_all = oracle.forward(th, st, n, e, F, L)
    keys = exact._keys(st)
    index = {int(k): a for a, k in enumerate(keys)}
    fn = lambda c: lp_all[[index[int(k)] for k in exact._keys(np.asarray(c))]]
    return n, e, st, lp_all, index, fn


def test_sampler_conserves_sz_and_tracks_logpsi():
    n, e, st, lp_all, index, fn = _setup()
    s0 = w.random_sz0_spins(64, n, 1)
    s, lp, acc = oracle.metropolis_sweeps(fn, s0, fn(s0), e, 3, seed=7)
    assert np.all(s.sum(1) == 0)
    assert np.array_equal(lp, fn(s))
    assert acc.max() <= 3 * n and acc.sum() > 0


def test_sampler_counter_continuation_and_determinism():
    n, e, st, lp_all, index, fn = _setup()
    s0 = w.random_sz0_spins(16, n, 2)
    a = oracle.metropolis_sweeps(fn, s0, fn(s0), e, 2, seed=9, counter_base=100)
    b1 = oracle.metropolis_sweeps(fn, s0, fn(s0), e, 1, seed=9, counter_base=100)
    b2 = oracle.metropolis_sweeps(fn, b1[0], b1[1], e, 1, seed=9, counter_base=100 + n)
    assert np.array_equal(a[0], b2[0]) and np.array_equal(a[2], b1[2] + b2[2])
    c = oracle.metropolis_sweeps(fn, s0, fn(s0), e, 2, seed=10, counter_base=100)
    assert not np.array_equal(a[0], c[0])


def test_transition_matrix_detailed_balance():
    # the proposal (uniform bond, identity on aligned bonds) is symmetric, and the
    # acceptance min(1, |psi'/psi|^2) then satisfies detailed balance for |psi|^2
    n, e, st, lp_all, index, fn = _setup()
    C = len(st)
    T = np.zeros((C, C))
    for a, s in enumerate(st):
        for i, j in e:
            if s[i] == s[j]:
                T[a, a] += 1 / len(e)
                continue
            t = s.copy()
            t[i], t[j] = s[j], s[i]
            b = index[int(exact._keys(t[None])[0])]
            acc = min(1.0, np.exp(2 * (lp_all[b, 0] - lp_all[a, 0])))
            T[a, b] += acc / len(e)
            T[a, a] += (1 - acc) / len(e)
    pi = np.exp(2 * (lp_all[:, 0] - lp_all[:, 0].max()))
    pi /= pi.sum()
    F_ = pi[:, None] * T
    assert np.allclose(F_, F_.T, atol=1e-15)
    assert np.allclose(pi @ T, pi, atol=1e-15)


@pytest.mark.slow
def test_sampler_histogram_matches_psi_squared():
    n, e, st, lp_all, index, fn = _setup(seed=8)
    pi = np.exp(2 * (lp_all[:, 0] - lp_all[:, 0].max()))
    pi /= pi.sum()
    s = w.random_sz0_spins(4000, n, 3)
    s, lp, _ = oracle.metropolis_sweeps(fn, s, fn(s), e, 20, seed=4)      # burn-in
    counts = np.zeros(len(st))
    for k in range(4):
        s, lp, _ = oracle.metropolis_sweeps(fn, s, lp, e, 5, seed=4, counter_base=(20 + 5 * k) * n)
        idx = [index[int(q)] for q in exact._keys(s)]
        counts += np.bincount(idx, minlength=len(st))
    # pool states into 30 bins of comparable probability for a valid chi-square
    order = np.argsort(pi)
    bins = np.array_split(order, 30)
    obs = np.array([counts[b].sum() for b in bins])
    exp_ = np.array([pi[b].sum() for b in bins]) * counts.sum()
    # snapshots 5 sweeps apart are close to independent at 12 sites; allow a margin
    chi2 = np.sum((obs - exp_) ** 2 / exp_)
    assert chi2 < sst.chi2.ppf(1 - 1e-4, 29) * 1.5


def test_sample_mean_energy_matches_exact():
    n, e, st, lp_all, index, fn = _setup(seed=8)
    Hm = exact.heisenberg_matrix(st, e)
    psi = exact.psi_from_logpsi(lp_all)
    Ev = exact.variational_energy(psi, Hm)
    s = w.random_sz0_spins(3000, n, 13)
    s, lp, _ = oracle.metropolis_sweeps(fn, s, fn(s), e, 25, seed=21)
    El = oracle.local_energy_generic(fn, s, e).real
    se = El.std() / np.sqrt(len(El))
    assert abs(El.mean() - Ev) < 5 * se
