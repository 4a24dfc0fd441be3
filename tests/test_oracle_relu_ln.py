"""Pins of the paper's own nonlinearity (Section 2: ReLU followed by a layer
normalisation) in the oracle: its hand-derived reverse pass against central
differences, the ISGO gradient against the exact variational energy, closed forms
of the zero rows, and the symmetries of the ansatz."""
import numpy as np
import pytest

import oracle
from oracle import exact, hcb
from oracle.gna import LN_EPS
import workloads as w


def _fd(f, th, h=1e-6):
    g = np.zeros_like(th)
    for k in range(th.size):
        e = np.zeros_like(th)
        e[k] = h * max(1.0, abs(th[k]))
        g[k] = (f(th + e) - f(th - e)) / (2 * e[k])
    return g


@pytest.mark.parametrize("tied", [True, False])
def test_vjp_matches_central_differences(tied):
    n, e = w.erdos_renyi_connected(10, 0.35, 2)
    F, L = 4, 2
    th = w.glorot_theta(F, L, tied, seed=4, weight_scale=1.5, bias_std=0.5)
    s = w.random_spins(5, n, 6)
    cot = np.random.default_rng(1).normal(size=(5, 2))
    g = oracle.logpsi_vjp(th, s, cot, n, e, F, L, tied, act_fn="relu_ln")
    fd = _fd(lambda t: np.sum(cot * oracle.forward(t, s, n, e, F, L, tied, act="relu_ln")), th)
    assert np.max(np.abs(g - fd)) < 1e-6 * max(1, np.max(np.abs(fd)))


def test_isgo_with_exact_weights_is_exact_gradient():
    # hard-core bosons (the workload the paper trains with this nonlinearity)
    n, e = w.kagome(2, 2)
    F, L = 4, 2
    th = w.glorot_theta(F, L, True, seed=1, weight_scale=1.5, bias_std=0.3, real_head=True)
    occ = hcb.occupations(n, n // 2)
    st = (2 * occ.astype(np.int64) - 1).astype(np.int8)
    Hb = hcb.hcb_matrix(occ, e, 0.5, 1.0)
    jz, jxy, hb_, cb = hcb.spin_couplings(0.5, 1.0)
    Ev = lambda t: exact.variational_energy(
        exact.psi_from_logpsi(oracle.forward(t, st, n, e, F, L, act="relu_ln")), Hb)
    lp = oracle.forward(th, st, n, e, F, L, act="relu_ln")
    wgt = np.exp(2 * (lp[:, 0] - lp[:, 0].max()))
    g, stats, E = oracle.isgo_grad(th, st, lp, n, e, F, L, counts=wgt, jz=jz, jxy=jxy, hb=hb_, cb=cb,
                                   act="relu_ln")
    assert abs(stats["e_re"] - Ev(th)) < 1e-10
    fd = _fd(Ev, th, h=1e-5)
    assert np.max(np.abs(g - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))


def test_rows_are_normalised():
    # every node's embedding has mean 0 over F and mean square var/(var + eps) <= 1
    n, e = w.kagome(2, 2)
    F, L = 8, 3
    th = w.glorot_theta(F, L, True, seed=3, weight_scale=2.0, bias_std=0.3)
    s = w.random_sz0_spins(4, n, 2)
    _, keep = oracle.forward(th, s, n, e, F, L, keep=True, act="relu_ln")
    for H, (y, r) in zip(keep["H"], keep["aux"]):
        assert np.max(np.abs(H.mean(axis=-1))) < 1e-13
        var = y.var(axis=-1)
        assert np.max(np.abs((H ** 2).mean(axis=-1) - var / (var + LN_EPS))) < 1e-12


def test_all_negative_preactivations_give_zero_rows():
    # a large negative bias switches every unit off: H = 0 after each layer, so only the
    # one-hot counts reach the readout (closed form)
    n, e = w.triangular(3, 4)
    F, L = 6, 2
    th = w.glorot_theta(F, L, True, seed=5)
    sl = w.param_slices(F, L, True)
    th[sl["b_e"][0]:sl["b_e"][1]] = -50.0
    th[sl["b"][0]:sl["b"][1]] = -50.0
    s = w.random_spins(6, n, 7)
    out = oracle.forward(th, s, n, e, F, L, act="relu_ln")
    p = oracle.unpack_theta(th, F, L)
    up = (s > 0).sum(axis=1)
    ref_a = p["v_a"][F] * (n - up) + p["v_a"][F + 1] * up + p["c_a"]
    ref_p = p["v_p"][F] * (n - up) + p["v_p"][F + 1] * up + p["c_p"]
    assert np.allclose(out[:, 0], ref_a, atol=1e-12) and np.allclose(out[:, 1], ref_p, atol=1e-12)


@pytest.mark.parametrize("kind", ["kagome", "triangular"])
def test_torus_translation_invariance(kind):
    if kind == "kagome":
        a, b = 4, 4
        n, e = w.kagome(a, b)
        shift = lambda s: s.reshape(-1, b, a, 3)[:, :, np.r_[1:a, 0], :].reshape(s.shape[0], -1)
    else:
        a, b = 4, 3
        n, e = w.triangular(a, b)
        shift = lambda s: s.reshape(-1, b, a)[:, :, np.r_[1:a, 0]].reshape(s.shape[0], -1)
    F, L = 5, 3
    th = w.glorot_theta(F, L, True, seed=8, weight_scale=1.5, bias_std=0.3)
    s = w.random_spins(4, n, 9)
    o1 = oracle.forward(th, s, n, e, F, L, act="relu_ln")
    o2 = oracle.forward(th, shift(s), n, e, F, L, act="relu_ln")
    assert np.allclose(o1, o2, atol=1e-12)


def test_three_aggregation_formulations_agree():
    n, e = w.erdos_renyi_connected(20, 0.2, 1)
    F, L = 5, 3
    th = w.glorot_theta(F, L, True, seed=2, weight_scale=1.5, bias_std=0.3)
    s = w.random_spins(4, n, 3)
    outs = [oracle.forward(th, s, n, e, F, L, formulation=f, act="relu_ln") for f in ("dense", "sparse", "edges")]
    assert np.allclose(outs[0], outs[1], atol=1e-13) and np.allclose(outs[0], outs[2], atol=1e-13)
