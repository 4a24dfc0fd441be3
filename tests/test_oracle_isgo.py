"""Pins for the reverse pass and the ISGO gradient (Eq. 2, 3)."""
import numpy as np
import pytest

import oracle
import workloads as w
from oracle import exact


def _fd(f, x, h=1e-5):
    g = np.zeros_like(x)
    for k in range(x.size):
        hk = h * max(1.0, abs(x[k]))
        xp, xm = x.copy(), x.copy()
        xp[k] += hk
        xm[k] -= hk
        g[k] = (f(xp) - f(xm)) / (2 * hk)
    return g


@pytest.mark.parametrize("tied", [True, False])
def test_vjp_matches_central_differences(tied):
    n, e = w.erdos_renyi_connected(10, 0.35, 2)
    F, L = 3, 2
    th = w.glorot_theta(F, L, tied, seed=4, weight_scale=1.5, bias_std=0.5)
    s = w.random_spins(5, n, 6)
    cot = np.random.default_rng(1).normal(size=(5, 2))
    g = oracle.logpsi_vjp(th, s, cot, n, e, F, L, tied)
    fd = _fd(lambda t: np.sum(cot * oracle.forward(t, s, n, e, F, L, tied)), th)
    assert np.max(np.abs(g - fd)) < 1e-7 * max(1, np.max(np.abs(fd)))


def _exact_setup(F=4, L=2, seed=0, graph="kagome"):
    if graph == "kagome":
        n, e = w.kagome(2, 2)
    else:
        n, e = w.triangular(3, 4)
    th = w.glorot_theta(F, L, True, seed=seed, weight_scale=1.5, bias_std=0.3)
    st = exact.enumerate_sz0(n)
    Hm = exact.heisenberg_matrix(st, e)
    return n, e, th, st, Hm, F, L


def _Ev(th, st, Hm, n, e, F, L):
    return exact.variational_energy(exact.psi_from_logpsi(oracle.forward(th, st, n, e, F, L)), Hm)


@pytest.mark.parametrize("graph", ["kagome", "triangular"])
def test_isgo_with_exact_weights_is_exact_gradient(graph):
    # samples = every state with count |psi|^2: the estimator becomes the exact
    # derivative of E_v = <psi|H|psi>/<psi|psi>, compared with its central difference
    n, e, th, st, Hm, F, L = _exact_setup(graph=graph)
    lp = oracle.forward(th, st, n, e, F, L)
    cnt = np.exp(2 * (lp[:, 0] - lp[:, 0].max()))
    g, stats, El = oracle.isgo_grad(th, st, lp, n, e, F, L, counts=cnt)
    fd = _fd(lambda t: _Ev(t, st, Hm, n, e, F, L), th)
    assert np.max(np.abs(g - fd)) < 2e-7 * np.max(np.abs(fd))
    assert stats["e_re"] == pytest.approx(_Ev(th, st, Hm, n, e, F, L), abs=1e-12)
    assert abs(stats["e_im"]) < 1e-12


def test_importance_identity_reweights_old_samples():
    # the exact old distribution reweighted to a new theta gives the new exact gradient
    n, e, th0, st, Hm, F, L = _exact_setup(seed=1)
    th1 = th0 + 0.05 * np.random.default_rng(3).normal(size=th0.size)
    lp0 = oracle.forward(th0, st, n, e, F, L)
    lp1 = oracle.forward(th1, st, n, e, F, L)
    cnt0 = np.exp(2 * (lp0[:, 0] - lp0[:, 0].max()))
    cnt1 = np.exp(2 * (lp1[:, 0] - lp1[:, 0].max()))
    g_re, s_re, _ = oracle.isgo_grad(th1, st, lp0, n, e, F, L, counts=cnt0)
    g_ex, s_ex, _ = oracle.isgo_grad(th1, st, lp1, n, e, F, L, counts=cnt1)
    assert np.max(np.abs(g_re - g_ex)) < 1e-12 * max(1, np.max(np.abs(g_ex)))
    assert s_re["e_re"] == pytest.approx(s_ex["e_re"], abs=1e-12)


def test_constant_log_derivative_components_vanish():
    # in S_z = 0 the one-hot counts in z and the head biases give a constant
    # O = d log psi/d theta, whose centred contribution is zero
    n, e, th, st, Hm, F, L = _exact_setup(seed=2)
    s = w.random_sz0_spins(64, n, 4)
    lp = oracle.forward(th, s, n, e, F, L)
    g, stats, _ = oracle.isgo_grad(th, s, lp, n, e, F, L)
    P = g.size
    sz = F + 2
    idx = [P - 2 * (sz + 1) + F, P - 2 * (sz + 1) + F + 1, P - sz - 2,       # v_a[F:F+2], c_a
           P - sz - 1 + F, P - sz - 1 + F + 1, P - 1]                        # v_p[F:F+2], c_p
    assert np.max(np.abs(g[idx])) < 1e-13
    assert np.max(np.abs(g)) > 1e-4


def test_stats_at_old_theta_reduce_to_plain_average():
    n, e, th, st, Hm, F, L = _exact_setup(seed=3)
    s = w.random_sz0_spins(40, n, 5)
    lp = oracle.forward(th, s, n, e, F, L)
    El = oracle.local_energy(th, s, n, e, F, L)
    stats, cot = oracle.isgo_stats(lp, lp, El)
    assert stats["ess"] == pytest.approx(40, rel=1e-14)
    assert stats["e_re"] == pytest.approx(El.real.mean(), rel=1e-13)
    assert stats["var"] == pytest.approx(np.mean(np.abs(El - El.mean()) ** 2), rel=1e-12)
    assert np.allclose(cot[:, 0], 2 / 40 * (El.real - El.real.mean()), atol=1e-14)
    # duplicates grouped with counts give the same statistics as the expanded batch
    stats2, _ = oracle.isgo_stats(np.repeat(lp, 3, 0), np.repeat(lp, 3, 0), np.repeat(El, 3))
    stats3, _ = oracle.isgo_stats(lp, lp, El, counts=np.full(40, 3.0))
    assert stats2["e_re"] == pytest.approx(stats3["e_re"], rel=1e-14)


def test_shift_makes_weights_overflow_safe():
    old = np.zeros((3, 2))
    new = np.array([[400.0, 0], [401.0, 0], [399.0, 0]])
    stats, cot = oracle.isgo_stats(old, new, np.array([1.0, 2.0, 3.0], complex))
    w_ = np.exp(np.array([0.0, 2.0, -2.0]))
    assert stats["e_re"] == pytest.approx(np.sum(w_ * [1, 2, 3]) / w_.sum(), rel=1e-14)
    assert stats["finite"]
    assert stats["shift"] == 802.0


def test_sgd_step_descends():
    n, e, th, st, Hm, F, L = _exact_setup(seed=4)
    lp = oracle.forward(th, st, n, e, F, L)
    cnt = np.exp(2 * (lp[:, 0] - lp[:, 0].max()))
    g, _, _ = oracle.isgo_grad(th, st, lp, n, e, F, L, counts=cnt)
    th2 = oracle.sgd_update(th, g, 1e-3)
    assert _Ev(th2, st, Hm, n, e, F, L) < _Ev(th, st, Hm, n, e, F, L)
