"""The sampling-iteration loop of Section 3 through the library: grouped duplicates
give the same trajectory as the full batch, a run resumed from a checkpoint is the
uninterrupted run, and parameters trained on 12 sites start larger lattices
(Section 4.2's transfer) at 108 and 432 sites, the transferred ansatz checked
against the oracle on each."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import hcb
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _ctx(n, e, F, L, prec, B, mode="incremental"):
    from paper_2011_12453_amd import GNA
    print(f"[gpu] vmc ctx N={n} F={F} L={L} {prec} {mode} B={B}", file=sys.stderr, flush=True)
    return GNA(n, e, F, L, tied=True, precision=prec, max_batch=B, device=DEV, eloc_mode=mode)


def _start(n, F, L, B, seed):
    theta = torch.from_numpy(w.glorot_theta(F, L, True, seed=seed, real_head=True)).to(DEV)
    spins = torch.from_numpy(w.random_sz0_spins(B, n, seed + 1000)).to(DEV)
    return theta, spins


def test_grouped_loop_follows_the_full_batch():
    from paper_2011_12453_amd.vmc import isgo_vmc
    n, e = w.kagome(2, 2)
    F, L, B = 16, 2, 512
    out = {}
    for group in (False, True):
        g = _ctx(n, e, F, L, "fp64", B)
        g.set_hard_core_bosons(0.5, 1.0)
        th, sp = _start(n, F, L, B, 3)
        hist, cb = isgo_vmc(g, th, sp, n_iters=3, n_updates=4, lr=0.05, seed=7, group=group)
        out[group] = (hist, th.cpu().numpy(), sp.cpu().numpy(), cb)
        g.close()
    (hf, tf, sf, cf), (hg, tg, sg, cg) = out[False], out[True]
    rows = [h["rows"] for h in hg]
    print(f"[gpu] grouped loop: rows per update {rows} of {B}", file=sys.stderr, flush=True)
    assert max(rows) < B and cf == cg and len(hf) == len(hg)
    for a, b in zip(hf, hg):
        assert abs(a["energy_per_site"] - b["energy_per_site"]) < 1e-10
        assert abs(a["variance"] - b["variance"]) < 1e-9 * max(1.0, a["variance"])
    assert np.max(np.abs(tf - tg)) < 1e-10 and np.array_equal(sf, sg)


def test_resume_from_checkpoint_is_the_uninterrupted_run(tmp_path):
    from paper_2011_12453_amd.vmc import isgo_vmc, load_checkpoint
    n, e = w.kagome(2, 2)
    F, L, B = 16, 2, 256
    ck = str(tmp_path / "ck.npz")
    g = _ctx(n, e, F, L, "fp32", B)
    g.set_hard_core_bosons(0.5, 1.0)
    th, sp = _start(n, F, L, B, 4)
    h_all, cb_all = isgo_vmc(g, th, sp, n_iters=4, n_updates=3, lr=0.05, seed=9, group=True)
    th2, sp2 = _start(n, F, L, B, 4)
    h1, _ = isgo_vmc(g, th2, sp2, n_iters=2, n_updates=3, lr=0.05, seed=9, group=True, checkpoint=ck)
    st = load_checkpoint(ck, g)
    assert st["iteration"] == 2
    h2, cb2 = isgo_vmc(g, st["theta"], st["spins"], n_iters=2, n_updates=3, lr=0.05, seed=9, group=True,
                       burn_in=0, counter_base=st["counter"], start_iter=st["iteration"])
    g.close()
    assert cb2 == cb_all
    assert torch.equal(st["theta"], th) and torch.equal(st["spins"], sp)   # bitwise: deterministic kernels
    assert [h["energy_per_site"] for h in h1 + h2] == [h["energy_per_site"] for h in h_all]


def test_transfer_from_12_sites():
    from paper_2011_12453_amd.vmc import isgo_vmc, transfer_theta
    F, L = 16, 2
    n12, e12 = w.kagome(2, 2)
    g12 = _ctx(n12, e12, F, L, "fp32", 1024)
    g12.set_hard_core_bosons(0.5, 1.0)
    th, sp = _start(n12, F, L, 1024, 0)
    isgo_vmc(g12, th, sp, n_iters=30, n_updates=5, lr=0.1, n_sweeps=2, seed=17, group=True)
    jz, jxy, hb_, cb = hcb.spin_couplings(0.5, 1.0)
    # 108 and 432 sites: energy per site at the transferred and at a fresh start,
    # same chains, and the transferred ansatz against the oracle on sampled rows
    for cells in (6, 12):
        n, e = w.kagome(cells, cells)
        B = 512
        res = {}
        for name in ("fresh", "transferred"):
            g = _ctx(n, e, F, L, "fp32", B)
            g.set_hard_core_bosons(0.5, 1.0)
            t0, s0 = _start(n, F, L, B, 1)
            if name == "transferred":
                t0 = transfer_theta(th, g12, g)
            hist, _ = isgo_vmc(g, t0, s0, n_iters=1, n_updates=1, lr=0.0, n_sweeps=4, burn_in=20, seed=3)
            res[name] = hist[0]["energy_per_site"]
            if name == "transferred":
                rows = s0[:3].contiguous()
                el, _ = g.local_energy(t0, rows)
                lp = g.logpsi(t0, rows).cpu().numpy()
                rows = rows.cpu().numpy()
                ref = oracle.local_energy(t0.cpu().numpy(), rows, n, e, F, L, jz=jz, jxy=jxy, hb=hb_, cb=cb)
                lp_ref = oracle.logpsi(t0.cpu().numpy(), rows, n, e, F, L)
                el = el.cpu().numpy()
                err = np.max(np.abs(el[:, 0] - ref.real) + np.abs(el[:, 1] - ref.imag)) / np.max(np.abs(ref))
                print(f"[gpu] transfer 12 -> {n} sites: E_loc rel {err:.2e}, log psi abs "
                      f"{np.max(np.abs(lp - lp_ref)):.2e}", file=sys.stderr, flush=True)
                assert err < 1e-5 and np.max(np.abs(lp - lp_ref)) < 1e-3
            g.close()
        print(f"[gpu] transfer 12 -> {n} sites: energy per site fresh {res['fresh']:.5f}, "
              f"transferred {res['transferred']:.5f}", file=sys.stderr, flush=True)
        assert res["transferred"] < res["fresh"]
    g12.close()
