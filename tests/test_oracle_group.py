"""Pins of the oracle's grouping of duplicated states (Section 3): a hand-checked
example, reconstruction and multiplicity identities, NumPy's own row-unique as an
independent routine, and the invariance of the ISGO estimates (energy, variance,
gradient) under grouping."""
import numpy as np

import oracle
import workloads as w


def test_hand_example():
    a, b, c = [1, -1, 1, -1], [-1, 1, 1, -1], [1, 1, -1, -1]
    s = np.array([a, b, a, c, b, a], dtype=np.int8)
    u, n, idx = oracle.group_duplicates(s)
    assert u.tolist() == [a, b, c]
    assert n.tolist() == [3.0, 2.0, 1.0]
    assert idx.tolist() == [0, 1, 0, 2, 1, 0]


def test_empty_and_all_distinct_and_all_equal():
    u, n, idx = oracle.group_duplicates(np.zeros((0, 6), np.int8))
    assert u.shape == (0, 6) and n.shape == (0,) and idx.shape == (0,)
    s = w.random_sz0_spins(1, 12, 3)
    u, n, idx = oracle.group_duplicates(np.repeat(s, 7, axis=0))
    assert u.shape == (1, 12) and n.tolist() == [7.0]
    states = oracle.exact.enumerate_sz0(8)
    u, n, idx = oracle.group_duplicates(states)
    assert np.array_equal(u, states) and np.all(n == 1)


def _batch_with_duplicates(B, n, seed):
    rng = np.random.default_rng(seed)
    pool = w.random_sz0_spins(max(2, B // 4), n, seed)
    return pool[rng.integers(0, pool.shape[0], size=B)]


def test_identities_and_numpy_unique():
    s = _batch_with_duplicates(500, 12, 1)
    u, n, idx = oracle.group_duplicates(s)
    assert np.array_equal(u[idx], s)
    assert np.array_equal(n, np.bincount(idx).astype(float)) and n.sum() == len(s)
    # first occurrences in increasing order
    first = np.array([np.flatnonzero(idx == g)[0] for g in range(len(u))])
    assert np.all(np.diff(first) > 0)
    # the same multiset of (row, count) as NumPy's lexicographic row-unique
    ru, rc = np.unique(s, axis=0, return_counts=True)
    mine = sorted((row.tobytes(), int(k)) for row, k in zip(u, n))
    ref = sorted((row.tobytes(), int(k)) for row, k in zip(ru, rc))
    assert mine == ref


def test_isgo_estimates_are_invariant_under_grouping():
    # Eq. 3 with multiplicities: the same weighted sums over fewer rows
    n, e = w.kagome(2, 2)
    F, L = 4, 2
    th_old = w.glorot_theta(F, L, True, seed=2, weight_scale=1.5, bias_std=0.3)
    th_new = th_old + 0.05 * np.random.default_rng(3).normal(size=th_old.size)
    s = _batch_with_duplicates(300, n, 4)
    lp_old = oracle.logpsi(th_old, s, n, e, F, L)
    u, cnt, idx = oracle.group_duplicates(s)
    first = np.array([np.flatnonzero(idx == g)[0] for g in range(len(u))])
    g_full, st_full, _ = oracle.isgo_grad(th_new, s, lp_old, n, e, F, L)
    g_grp, st_grp, _ = oracle.isgo_grad(th_new, u, lp_old[first], n, e, F, L, counts=cnt)
    assert len(u) < len(s)
    assert abs(st_full["e_re"] - st_grp["e_re"]) < 1e-12 * abs(st_full["e_re"])
    assert abs(st_full["e_im"] - st_grp["e_im"]) < 1e-12
    assert abs(st_full["var"] - st_grp["var"]) < 1e-12 * st_full["var"]
    assert np.max(np.abs(g_full - g_grp)) < 1e-12 * np.max(np.abs(g_full))
