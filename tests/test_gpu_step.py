"""The device-resident step (gna_step): equal to its parts called one by one, and
replayable from a HIP graph (captured through torch.cuda.graph on the library's
stream) with results identical to eager execution on every replay."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _ctx(n, e, F, L, prec, B, mode, act="tanh"):
    from paper_2011_12453_amd import GNA
    print(f"[gpu] step ctx N={n} F={F} L={L} {prec} {mode} {act} B={B}", file=sys.stderr, flush=True)
    return GNA(n, e, F, L, tied=True, precision=prec, max_batch=B, device=DEV, eloc_mode=mode, activation=act)


def _state(n, F, L, B, seed):
    theta = torch.from_numpy(w.glorot_theta(F, L, True, seed=seed, weight_scale=1.5, bias_std=0.3)).to(DEV)
    spins = torch.from_numpy(w.random_sz0_spins(B, n, seed + 100)).to(DEV)
    return theta, spins


@pytest.mark.parametrize("mode,prec,act", [("full", "fp64", "tanh"), ("incremental", "fp64", "tanh"),
                                           ("incremental", "bf16_1x", "tanh"), ("incremental", "bf16", "tanh"),
                                           ("incremental", "fp32", "relu_ln"), ("full", "fp32", "relu_ln")])
def test_step_equals_its_parts(mode, prec, act):
    # the step reuses the sweep's final log psi and (incremental) its planes as the
    # ISGO update's base pass: bitwise the same as calling the parts one by one
    n, e = w.kagome(6, 6)
    F, L, B, seed, lr = 32, 4, 32, 7, 1e-3
    g = _ctx(n, e, F, L, prec, B, mode, act)
    th1, sp1 = _state(n, F, L, B, 3)
    th2, sp2 = th1.clone(), sp1.clone()
    lp1 = torch.empty(B, 2, dtype=torch.float64, device=DEV)
    counter = torch.zeros(1, dtype=torch.int64, device=DEV)
    for k in range(2):
        grad1, stats1, el1, acc1 = g.step(th1, sp1, lp1, 1, seed, counter, lr)
        lp2 = g.logpsi(th2, sp2)
        acc2 = g.metropolis_sweep(th2, sp2, lp2, n_sweeps=1, seed=seed, counter_base=k * n)
        grad2, stats2, el2 = g.isgo_grad(th2, sp2, lp2)
        g.sgd_update(th2, grad2, lr)
        torch.cuda.synchronize()
        assert torch.equal(sp1, sp2) and torch.equal(acc1, acc2) and torch.equal(lp1, lp2)
        assert torch.equal(grad1, grad2) and torch.equal(stats1, stats2) and torch.equal(th1, th2)
    assert int(counter.item()) == 2 * n
    # the sampled configurations are the oracle's trajectory (FP64 decisions)
    g.close()


@pytest.mark.parametrize("mode,prec", [("incremental", "bf16"), ("full", "fp32"), ("incremental", "fp64"),
                                       ("incremental", "bf16_1x")])
def test_step_graph_replay_matches_eager(mode, prec):
    n, e = w.kagome(6, 6)
    F, L, B, seed, lr = 32, 4, 48, 11, 2e-3
    g = _ctx(n, e, F, L, prec, B, mode)
    P = g.num_params
    th0, sp0 = _state(n, F, L, B, 5)
    # eager reference: three steps
    th_e, sp_e = th0.clone(), sp0.clone()
    lp_e = torch.empty(B, 2, dtype=torch.float64, device=DEV)
    cnt_e = torch.zeros(1, dtype=torch.int64, device=DEV)
    ref = []
    for k in range(3):
        grad, stats, el, acc = g.step(th_e, sp_e, lp_e, 1, seed, cnt_e, lr)
        torch.cuda.synchronize()
        ref.append(tuple(t.clone() for t in (th_e, sp_e, lp_e, grad, stats, el, acc)))
    # graph: static buffers, one captured step, replayed three times
    th_g, sp_g = th0.clone(), sp0.clone()
    lp_g = torch.empty(B, 2, dtype=torch.float64, device=DEV)
    cnt_g = torch.zeros(1, dtype=torch.int64, device=DEV)
    grad_g = torch.empty(P, dtype=torch.float64, device=DEV)
    stats_g = torch.empty(8, dtype=torch.float64, device=DEV)
    el_g = torch.empty(B, 2, dtype=torch.float64, device=DEV)
    acc_g = torch.empty(B, dtype=torch.int32, device=DEV)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.set_stream(torch.cuda.current_stream())
        g.step(th_g, sp_g, lp_g, 1, seed, cnt_g, lr, grad=grad_g, stats=stats_g, eloc=el_g, n_accept=acc_g)
    g.set_stream(torch.cuda.current_stream())
    other = torch.from_numpy(w.random_sz0_spins(B, n, 999)).to(DEV)
    for k in range(3):
        graph.replay()
        torch.cuda.synchronize()
        got = (th_g, sp_g, lp_g, grad_g, stats_g, el_g, acc_g)
        for a, b in zip(got, ref[k]):
            assert torch.equal(a, b), f"replay {k} differs from eager step {k}"
        # the program's own eager work between replays
        g.logpsi(th_g.clone(), other)
        torch.cuda.synchronize()
    assert int(cnt_g.item()) == 3 * n
    print(f"[gpu] graph replay {mode} {prec}: 3 replays identical to eager; E/site "
          f"{stats_g[0].item() / n:.6f}", file=sys.stderr, flush=True)
    g.close()


def test_step_sampler_matches_oracle_trajectory():
    # gna_step's sweep with the device counter is the oracle's Metropolis chain
    n, e = w.kagome(2, 2)
    F, L, B, seed = 16, 2, 16, 21
    g = _ctx(n, e, F, L, "fp64", B, "incremental")
    theta = w.glorot_theta(F, L, True, seed=3, weight_scale=2.0, bias_std=0.3)
    s0 = w.random_sz0_spins(B, n, 4)
    th, sp = torch.from_numpy(theta).to(DEV), torch.from_numpy(s0).to(DEV)
    lp = torch.empty(B, 2, dtype=torch.float64, device=DEV)
    counter = torch.tensor([5 * n], dtype=torch.int64, device=DEV)
    g.step(th, sp, lp, 2, seed, counter, 0.0)
    fn = lambda c: oracle.logpsi(theta, c, n, e, F, L)
    rs, rlp, racc = oracle.metropolis_sweeps(fn, s0, fn(s0), e, 2, seed=seed, counter_base=5 * n)
    assert np.array_equal(sp.cpu().numpy(), rs)
    assert np.max(np.abs(lp.cpu().numpy() - rlp)) < 1e-11
    g.close()


def test_autotune_keeps_results_and_is_cached():
    n, e = w.kagome(6, 6)
    F, L, B = 32, 4, 64
    th, sp = _state(n, F, L, B, 9)
    g1 = _ctx(n, e, F, L, "bf16", B, "incremental")
    el0, nev0 = g1.local_energy(th, sp)
    choice = g1.autotune(th, sp)
    info = g1.config_info()
    print(f"[gpu] autotune kagome108 bf16: {choice} -> {info}", file=sys.stderr, flush=True)
    assert info["jobs_in_flight"] == choice["jobs_in_flight"] >= 1
    assert info["waves"] == choice["waves"] and info["samples_per_xcd"] == choice["samples_per_xcd"]
    assert info["sweep_jobs_in_flight"] == choice["sweep_jobs_in_flight"] >= 1
    assert info["sweep_waves"] == choice["sweep_waves"] and choice["sweep_us_per_call"] > 0
    el1, nev1 = g1.local_energy(th, sp)
    # the shape changes only the order of the final FP64 sums
    scale = float(el0.abs().max())
    assert int(nev0.item()) == int(nev1.item())
    assert float((el1 - el0).abs().max()) < 1e-12 * scale
    # a later context of the same signature starts from the tuned shape
    g2 = _ctx(n, e, F, L, "bf16", B, "incremental")
    assert g2.config_info() == info
    el2, _ = g2.local_energy(th, sp)
    assert torch.equal(el2, el1)
    # and its sampler still takes the full sampler's decisions
    lp = g2.logpsi(th, sp)
    s_inc = sp.clone()
    acc_i = g2.metropolis_sweep(th, s_inc, lp.clone(), n_sweeps=1, seed=3)
    g3 = _ctx(n, e, F, L, "bf16", B, "full")
    s_full = sp.clone()
    acc_f = g3.metropolis_sweep(th, s_full, g3.logpsi(th, sp), n_sweeps=1, seed=3)
    assert torch.equal(s_inc, s_full) and torch.equal(acc_i, acc_f)
    for g in (g1, g2, g3):
        g.close()


def test_autotune_leaves_the_batch_alone():
    # the sweep is tuned on a copy: the caller's configurations do not move
    n, e = w.kagome(6, 6)
    th, sp = _state(n, 32, 4, 16, 4)
    before = sp.clone()
    g = _ctx(n, e, 32, 4, "fp32", 16, "incremental")
    g.autotune(th, sp)
    assert torch.equal(sp, before)
    g.close()


@pytest.mark.parametrize("which", ["eloc", "sweep", "both"])
def test_pinned_shapes_give_the_same_results(which):
    n, e = w.kagome(6, 6)
    F, L, B = 32, 4, 24
    th, sp = _state(n, F, L, B, 5)
    ref = _ctx(n, e, F, L, "bf16", B, "incremental")
    el_r, _ = ref.local_energy(th, sp)
    s_r = sp.clone()
    acc_r = ref.metropolis_sweep(th, s_r, ref.logpsi(th, sp), n_sweeps=1, seed=11)
    ref.close()
    g = _ctx(n, e, F, L, "bf16", B, "incremental")
    for jobs, waves, px in ((1, 8, 1), (2, 16, 2), (3, 6, 2)):
        g.set_shape(jobs, waves, px, which=which)
        info = g.config_info()
        # narrow variants are capped at the tiles the jobs have (4 per job here);
        # 16 names the one-tile-per-wave variant
        wv = waves if waves == 16 else min(waves, 4 * jobs)
        if which in ("eloc", "both"):
            assert (info["jobs_in_flight"], info["waves"], info["samples_per_xcd"]) == (jobs, wv, px)
        if which in ("sweep", "both"):
            assert (info["sweep_jobs_in_flight"], info["sweep_waves"]) == (jobs, wv)
        el, _ = g.local_energy(th, sp)
        assert float((el - el_r).abs().max()) < 1e-12 * float(el_r.abs().max())
        s1 = sp.clone()
        acc = g.metropolis_sweep(th, s1, g.logpsi(th, sp), n_sweeps=1, seed=11)
        assert torch.equal(s1, s_r) and torch.equal(acc, acc_r)
    # a tuned shape pinned again is the same shape
    tuned = g.autotune(th, sp)
    info = g.config_info()
    g.set_shape(tuned["jobs_in_flight"], tuned["waves"], tuned["samples_per_xcd"], which="eloc")
    g.set_shape(tuned["sweep_jobs_in_flight"], tuned["sweep_waves"], 1, which="sweep")
    assert g.config_info() == info
    g.close()


def test_set_shape_rejects_bad_shapes():
    from paper_2011_12453_amd.binding import GnaError
    n, e = w.kagome(6, 6)
    g = _ctx(n, e, 32, 4, "bf16", 8, "incremental")
    before = g.config_info()
    for args in ((-1, 8, 1), (0, 6, 1), (9, 8, 1), (2, 12, 1), (2, 8, 0), (8, 1, 1)):
        with pytest.raises(GnaError):
            g.set_shape(*args)
        assert g.config_info() == before
    g.close()
    f = _ctx(n, e, 32, 4, "bf16", 8, "full")
    with pytest.raises(GnaError):
        f.set_shape(2, 8, 1)
    f.close()


def test_autotune_full_mode_is_a_no_op():
    n, e = w.kagome(2, 2)
    th, sp = _state(n, 16, 2, 8, 1)
    g = _ctx(n, e, 16, 2, "fp32", 8, "full")
    assert g.autotune(th, sp)["jobs_in_flight"] == 0
    assert g.config_info()["eloc_mode"] == 0
    g.close()
