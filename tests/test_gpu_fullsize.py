"""GPU parity at the measured workload's own shape (432-site Kagome torus, 6 tied
layers of width 64, 2048 samples in one launch) with checks that a broken kernel
cannot pass, the reverse pass at F = 64, the chunked recompute of the reverse
pass, and invariances that need no oracle.

Discriminating measure.  With Glorot weights psi is close to uniform and every
local energy is close to |E|/4 (a constant psi gives exactly |E|/4), so the energy
per site alone cannot tell a correct kernel from one that returns
psi(s^ij)/psi(s) = 1.  These tests therefore also compare, sample by sample, the
off-diagonal part E_loc - |E|/4 = (1/2) sum_anti [psi(s^ij)/psi(s) - 1] (Section
3's E_x minus its constant-psi value), relative to its own size: a constant-psi
kernel scores exactly 1 there.  Rows are sampled from the batch the GPU evaluated
in one launch; the oracle evaluates them one by one on the same parameters.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
EPS_SITE = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3, "bf16_1x": 1e-3}
N_ROWS = 16
_ORACLE = {}


def _ctx(n, e, F, L, prec, B, mode="incremental", **kw):
    from paper_2011_12453_amd import GNA
    print(f"[gpu] fullsize ctx N={n} F={F} L={L} {prec} {mode} B={B} {kw}", file=sys.stderr, flush=True)
    return GNA(n, e, F, L, tied=True, precision=prec, max_batch=B, device=DEV, eloc_mode=mode, **kw)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _theta(F, L, kind, seed=0):
    if kind == "glorot":   # the workload's initialisation: Glorot-normal, zero biases
        return w.glorot_theta(F, L, True, seed=seed)
    # far from uniform psi: larger weights and random biases
    return w.glorot_theta(F, L, True, seed=seed, weight_scale=1.5, bias_std=0.3)


def _workload_432(kind):
    """Inputs of the 432-site workload and the oracle on N_ROWS sampled rows (cached)."""
    if kind not in _ORACLE:
        p = w.preset("kagome432_L6F64")
        n, e = p.build_graph()
        theta = _theta(p.n_features, p.n_layers, kind, p.theta_seed)
        spins = w.random_sz0_spins(p.batch, n, p.spin_seed)
        rows = np.sort(np.random.default_rng(11).choice(p.batch, size=N_ROWS, replace=False))
        print(f"[gpu] oracle 432-site {kind}: {N_ROWS} rows", file=sys.stderr, flush=True)
        lp_ref = oracle.logpsi(theta, spins[rows], n, e, p.n_features, p.n_layers)
        el_ref = oracle.local_energy(theta, spins[rows], n, e, p.n_features, p.n_layers)
        _ORACLE[kind] = (p, n, e, theta, spins, rows, lp_ref, el_ref)
    return _ORACLE[kind]


def _offdiag_err(got, ref, n_edges):
    """Per-sample |E_loc - E_ref| over the largest off-diagonal part |E_ref - |E|/4| of
    the rows (a constant-psi kernel scores 1 on the row where that part peaks)."""
    g = got[:, 0] + 1j * got[:, 1]
    return np.abs(g - ref) / np.max(np.abs(ref - n_edges / 4.0))


def _centred(lp):
    return lp - lp.mean(axis=0, keepdims=True)


# per-sample bounds.  log psi: FP32/FP64 absolute (|log psi| is O(10) here).  The
# BF16 modes store W in bfloat16, a fixed perturbation of the ansatz that shifts
# log psi by the same amount for every configuration up to a slowly varying part
# (0.17 at Glorot weights, 1.1 at the stress weights, measured): that shift cancels
# in every ratio psi(s')/psi(s) the method uses, so BF16 log psi is compared after
# removing its mean over the sampled rows, against a tenth of the reference's own
# spread over them.  E_loc: error over the largest off-diagonal part; FP32 carries
# ~1e-7 per operation over six layers, split BF16 ~16-bit activations with 8-bit
# weights (about 1% of the part, measured), both far below the 1 of a constant psi.
LP_TOL = {"fp64": 1e-10, "fp32": 2e-4}
OFF_TOL = {"fp64": 1e-9, "fp32": 1e-3, "bf16": 5e-2}


@pytest.mark.parametrize("kind", ["glorot", "stress"])
@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp64"])
def test_432_incremental_per_sample_parity(prec, kind):
    p, n, e, theta, spins, rows, lp_ref, el_ref = _workload_432(kind)
    g = _ctx(n, e, p.n_features, p.n_layers, prec, p.batch)
    th, sp = _dev(theta), _dev(spins)
    el, nev = g.local_energy(th, sp)
    lp = g.logpsi(th, sp)
    el, lp = el.cpu().numpy(), lp.cpu().numpy()
    g.close()
    assert int(nev.item()) == oracle.n_evals(spins, e)
    assert np.all(np.isfinite(el)) and np.all(np.isfinite(lp))
    lp_err = np.max(np.abs(lp[rows] - lp_ref))
    lp_cerr = np.max(np.abs(_centred(lp[rows]) - _centred(lp_ref)))
    lp_spread = np.max(np.abs(_centred(lp_ref)))
    off = _offdiag_err(el[rows], el_ref, len(e))
    site = abs(np.mean(el[rows, 0]) - np.mean(el_ref.real)) / n / max(abs(np.mean(el_ref.real)) / n, 1e-2)
    offpart = np.abs(el_ref - len(e) / 4.0)
    print(f"[gpu] 432 {prec} {kind}: logpsi abs {lp_err:.2e}, centred {lp_cerr:.2e} (spread {lp_spread:.2e}); "
          f"off-diagonal part {offpart.min():.3f}..{offpart.max():.3f}, err/part max {off.max():.2e} "
          f"median {np.median(off):.2e}; e/site rel {site:.2e}", file=sys.stderr, flush=True)
    if prec in LP_TOL:
        assert lp_err < LP_TOL[prec]
    else:
        assert lp_cerr < 0.1 * lp_spread
    assert off.max() < OFF_TOL[prec]
    assert site < EPS_SITE[prec]


def test_432_single_pass_bf16_is_reported_not_bounded():
    # single-pass BF16 (activations rounded to 8 bits) is the fast, coarse mode: its
    # per-sample off-diagonal error is of the order of the part itself at Glorot
    # weights, so it is held only to the constant-psi bound it must beat and to the
    # incremental = full identity; its measured errors are printed for the record
    p, n, e, theta, spins, rows, lp_ref, el_ref = _workload_432("stress")
    sub = spins[rows]
    out = {}
    for mode in ("incremental", "full"):
        g = _ctx(n, e, p.n_features, p.n_layers, "bf16_1x", N_ROWS, mode)
        el, _ = g.local_energy(_dev(theta), _dev(sub))
        out[mode] = el.cpu().numpy()
        g.close()
    assert np.max(np.abs(out["incremental"] - out["full"])) < 1e-12 * np.max(np.abs(el_ref))
    off = _offdiag_err(out["incremental"], el_ref, len(e))
    site = abs(np.mean(out["incremental"][:, 0]) - np.mean(el_ref.real)) / n / max(abs(np.mean(el_ref.real)) / n, 1e-2)
    print(f"[gpu] 432 bf16_1x stress: off-diagonal err/part max {off.max():.2e} median {np.median(off):.2e}; "
          f"e/site rel {site:.2e}", file=sys.stderr, flush=True)
    assert np.median(off) < 0.5



# ---------------------------------------------------------------------------
# reverse pass at F = 64 (the instantiation every benchmark step runs)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_vjp_F64_L6_matches_oracle(prec):
    n, e = w.kagome(6, 6)
    F, L = 64, 6
    theta = _theta(F, L, "stress", seed=4)
    spins = w.random_sz0_spins(8, n, 5)
    cot = np.random.default_rng(0).normal(size=(8, 2))
    g = _ctx(n, e, F, L, prec, 8)
    got = g.logpsi_vjp(_dev(theta), _dev(spins), _dev(cot)).cpu().numpy()
    g.close()
    ref = oracle.logpsi_vjp(theta, spins, cot, n, e, F, L)
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    emax = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"[gpu] vjp F=64 L=6 {prec}: rel norm {err:.2e}, rel max {emax:.2e}", file=sys.stderr, flush=True)
    # FP64 reverse pass for FP64, FP32 for the FP32 and BF16 modes
    assert emax < (1e-11 if prec == "fp64" else 1e-4)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_vjp_432_full_batch_launch(prec):
    # the whole 2048-sample batch in one call, as the benchmark's step runs it;
    # cotangents vanish outside N_ROWS sampled rows, so the result is the oracle's
    # reverse pass over those rows
    p, n, e, theta, spins, rows, _, _ = _workload_432("stress")
    cot = np.zeros((p.batch, 2))
    cot[rows] = np.random.default_rng(3).normal(size=(N_ROWS, 2))
    g = _ctx(n, e, p.n_features, p.n_layers, prec, p.batch)
    got = g.logpsi_vjp(_dev(theta), _dev(spins), _dev(cot)).cpu().numpy()
    g.close()
    ref = oracle.logpsi_vjp(theta, spins[rows], cot[rows], n, e, p.n_features, p.n_layers)
    emax = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    print(f"[gpu] vjp 432 full batch {prec}: rel max {emax:.2e}", file=sys.stderr, flush=True)
    assert emax < 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_isgo_grad_F64_matches_oracle(prec):
    n, e = w.kagome(6, 6)
    F, L = 64, 4
    th_old = _theta(F, L, "stress", seed=6)
    th_new = th_old + 0.02 * np.random.default_rng(1).normal(size=th_old.size)
    spins = w.random_sz0_spins(48, n, 21)
    lp_old = oracle.logpsi(th_old, spins, n, e, F, L)
    for mode in ("full", "incremental"):
        g = _ctx(n, e, F, L, prec, 48, mode)
        grad, stats, _ = g.isgo_grad(_dev(th_new), _dev(spins), _dev(lp_old))
        grad, stats = grad.cpu().numpy(), stats.cpu().numpy()
        g.close()
        if mode == "full":
            rg, rs, _ = oracle.isgo_grad(th_new, spins, lp_old, n, e, F, L)
        err = np.max(np.abs(grad - rg)) / np.max(np.abs(rg))
        print(f"[gpu] isgo F=64 {prec} {mode}: grad rel {err:.2e}", file=sys.stderr, flush=True)
        assert err < {"fp64": 1e-10, "fp32": 1e-3}[prec]
        assert abs(stats[0] - rs["e_re"]) / n < {"fp64": 1e-10, "fp32": 1e-5}[prec] * max(abs(rs["e_re"]) / n, 1e-2)
        assert stats[6] == rs["n_evals"]


# ---------------------------------------------------------------------------
# recompute in chunks when the batch's activations exceed the budget
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("budget", [1, 600 << 10])
def test_chunked_recompute_equals_one_pass(prec, budget):
    # budget 1 byte: one sample per chunk (12 chunks); 600 KiB: a few samples each
    n, e = w.kagome(6, 6)
    F, L, B = 32, 4, 12
    theta = _theta(F, L, "stress", seed=9)
    spins = w.random_sz0_spins(B, n, 4)
    cot = np.random.default_rng(5).normal(size=(B, 2))
    lp_old = oracle.logpsi(theta - 0.01, spins, n, e, F, L)
    out = {}
    for b in (0, budget):
        g = _ctx(n, e, F, L, prec, B, "full", act_budget_bytes=b)
        vjp = g.logpsi_vjp(_dev(theta), _dev(spins), _dev(cot)).cpu().numpy()
        grad, _, _ = g.isgo_grad(_dev(theta), _dev(spins), _dev(lp_old))
        out[b] = (vjp, grad.cpu().numpy())
        g.close()
    (v0, g0), (v1, g1) = out[0], out[budget]
    ev = np.max(np.abs(v1 - v0)) / np.max(np.abs(v0))
    eg = np.max(np.abs(g1 - g0)) / np.max(np.abs(g0))
    print(f"[gpu] chunked recompute {prec} budget {budget}: vjp rel {ev:.2e} isgo rel {eg:.2e}", file=sys.stderr,
          flush=True)
    # same per-sample arithmetic; only the order of the per-workgroup sums differs
    tol = 1e-13 if prec == "fp64" else 1e-5
    assert ev < tol and eg < tol
    ref = oracle.logpsi_vjp(theta, spins, cot, n, e, F, L)
    assert np.max(np.abs(v1 - ref)) / np.max(np.abs(ref)) < (1e-11 if prec == "fp64" else 1e-4)


# ---------------------------------------------------------------------------
# invariances (no oracle): torus translations, and torch's gradient check
# ---------------------------------------------------------------------------
def _kagome_shift(l1, l2, dx, dy):
    """Site map of the translation by (dx, dy) cells on the l1 x l2 Kagome torus."""
    perm = np.empty(3 * l1 * l2, dtype=np.int64)
    for y in range(l2):
        for x in range(l1):
            for s in range(3):
                perm[3 * (x + l1 * y) + s] = 3 * ((x + dx) % l1 + l1 * ((y + dy) % l2)) + s
    return perm


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_torus_translation_invariance_432(prec):
    p = w.preset("kagome432_L6F64")
    n, e = p.build_graph()
    theta = _theta(p.n_features, p.n_layers, "stress", seed=2)
    s = w.random_sz0_spins(24, n, 77)
    batch = [s]
    for dx, dy in ((1, 0), (0, 1), (5, 7)):
        perm = _kagome_shift(12, 12, dx, dy)
        t = np.empty_like(s)
        t[:, perm] = s                      # spin of site i moves to site perm[i]
        batch.append(t)
    allsp = np.concatenate(batch)
    g = _ctx(n, e, p.n_features, p.n_layers, prec, len(allsp))
    lp = g.logpsi(_dev(theta), _dev(allsp)).cpu().numpy().reshape(4, 24, 2)
    el = g.local_energy(_dev(theta), _dev(allsp))[0].cpu().numpy().reshape(4, 24, 2)
    g.close()
    dlp = np.max(np.abs(lp[1:] - lp[0][None]))
    delo = np.max(np.abs(el[1:] - el[0][None]) / np.abs(el[0][None] - len(e) / 4.0).max(axis=-1, keepdims=True))
    print(f"[gpu] translation invariance 432 {prec}: logpsi abs {dlp:.2e}, E_loc rel {delo:.2e}", file=sys.stderr,
          flush=True)
    # the translated configuration is evaluated with another node order inside the
    # sums: equal up to rounding (the node rows themselves are computed identically)
    assert dlp < {"fp64": 1e-10, "fp32": 1e-4, "bf16": 1e-3}[prec]
    assert delo < {"fp64": 1e-9, "fp32": 1e-3, "bf16": 1e-2}[prec]


def test_logpsi_autograd_gradcheck():
    from paper_2011_12453_amd import LogPsi
    n, e = w.kagome(2, 2)
    F, L = 16, 2
    theta = _theta(F, L, "stress", seed=8)
    spins = _dev(w.random_sz0_spins(3, n, 4))
    g = _ctx(n, e, F, L, "fp64", 4, "full")
    th = _dev(theta).requires_grad_(True)
    ok = torch.autograd.gradcheck(lambda t: LogPsi.apply(g, t, spins), (th,), eps=1e-6, atol=1e-6, rtol=1e-5)
    g.close()
    assert ok
