#!/usr/bin/env python
"""Benchmark: log-psi evaluations per second inside the local energy, 432-site Kagome.

One step is one pass of the whole hot path over a batch of 2048 chains on the
12x12x3 Kagome torus (864 bonds, GCN with 6 tied layers of width 64):

    refresh log psi -> one Metropolis sweep (432 proposals per chain) ->
    ISGO update (log psi, E_loc over every exchanged configuration, weights,
    reverse pass) -> SGD update

``value`` = local-energy log-psi evaluations (the library's exact count) per
second of whole-step wall time, BF16 layer products (``--precision``; the other
precisions are timed on the local energy alone beside it, every one at the same
2048-sample batch, each with its error against the oracle).  The timed steps run
without per-kernel events; a separate profiled pass gives the per-kernel
durations (HIP events the library records on its stream) for the roofline
entries of the local-energy and sweep kernels.  The CPU baseline times the FP64
oracle on a bounded prefix of the same batch, and its outputs give the error
columns: energy per site, and per sample the off-diagonal part E_loc - |E|/4,
which a constant psi would get wrong (median of the per-sample error relative to
each sample's part, and the largest error relative to the largest part; a
constant psi scores 1 on both).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "log-psi evals/sec in E_loc (432-site Kagome), BF16 vs FP32 vs FP64 at stated err"
PEAK = {"bf16": 2.5e15, "bf16_1x": 2.5e15, "fp32": 157.3e12, "fp64": 78.6e12}   # MI355X dense MFMA, FLOP/s
HBM_PEAK = 8.0e12                                                                  # MI355X HBM3E, B/s
BOUND = {"fp64": 1e-10, "fp32": 1e-5, "bf16": 1e-3, "bf16_1x": 1e-3}              # energy per site, relative
LATTICE = {"kagome": "kagome torus", "triangular": "triangular torus", "er": "random graph G(n, p)"}


def flops_per_eval(n, n_edges, F, L):
    """Algorithmic FLOPs of one log-psi evaluation: per layer the [M|H] W product
    (2 N 2F F) and the aggregation (2 per stored adjacency entry per feature), plus
    the two-head readout.  tanh is not counted."""
    return L * (2 * n * 2 * F * F + 2 * (2 * n_edges) * F) + 2 * 2 * n * F


def balls(n, edges, L):
    """For each bond (i, j): the nested balls C_0 = {i, j}, C_l = C_{l-1} plus its
    neighbours, l = 0 .. L + 1 (graph distance <= l from the bond), and the degrees."""
    import numpy as np
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    deg = np.array([len(x) for x in adj])
    out = []
    for a, b in edges:
        bl = [{int(a), int(b)}]
        for _ in range(L + 1):
            nxt = set(bl[-1])
            for u in bl[-1]:
                nxt.update(adj[u])
            bl.append(nxt)
        out.append(bl)
    return out, deg


def ball_flops(n, edges, F, L):
    """Algorithmic FLOPs of one incremental evaluation for each bond: at layer l the
    message product of the ball C_{l-1} and the self product, aggregation and
    activation input of the ball C_l (C_0 = the bond, C_l = C_{l-1} plus neighbours),
    plus the two-head readout difference over C_L."""
    import numpy as np
    bl_all, deg = balls(n, edges, L)
    out = []
    for bl in bl_all:
        f = 0
        for l in range(1, L + 1):
            f += 2 * len(bl[l - 1]) * F * F + 2 * len(bl[l]) * F * F
            f += 2 * int(deg[list(bl[l])].sum()) * F
        f += 2 * 2 * len(bl[L]) * F
        out.append(f)
    return np.array(out, dtype=np.float64)


def ball_bytes(n, edges, F, L, acc_bytes):
    """Algorithmic HBM bytes of one Metropolis proposal on bond (i, j) in the
    receptive-field evaluation, per bond: (read, write).  Read: the stored rows of
    the unchanged configuration it combines with the recomputed ones (layer l: the
    layer input H^{l-1} of ring l = C_l minus C_{l-1} and the message product
    G^{l-1} of ring l+1, F values each) and the base readout partials of C_L (8
    values per node).  Written when the proposal is accepted: the new rows H^l of C_l
    (l < L), G^{l-1} of C_{l-1} (l = 1 .. L) and the readout partials of C_L."""
    import numpy as np
    bl_all, _ = balls(n, edges, L)
    rd, wr = [], []
    for bl in bl_all:
        r = 8 * len(bl[L])
        w_ = 8 * len(bl[L])
        for l in range(1, L + 1):
            r += F * (len(bl[l + 1]) - len(bl[l]))
            if l >= 2:
                r += F * (len(bl[l]) - len(bl[l - 1]))
            w_ += F * len(bl[l - 1])
            if l < L:
                w_ += F * len(bl[l])
        rd.append(r * acc_bytes)
        wr.append(w_ * acc_bytes)
    return np.array(rd, dtype=np.float64), np.array(wr, dtype=np.float64)


def source_hash() -> str:
    """sha256[:16] of the HIP sources, to tie stored counter readings to a build."""
    import hashlib
    d = os.path.join(ROOT, "paper_2011_12453_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_of(prof: dict, names) -> str:
    """The first of `names` (local-energy or sweep kernels of a mode, pipelined or
    grouped) that ran in a profile."""
    for nm in names:
        if prof.get(nm, (0, 0.0))[0]:
            return nm
    return names[0]


ELOC_KERNELS = {"incremental": ("k_eloc_pipe", "k_eloc_inc"), "full": ("k_eloc",)}
SWEEP_KERNELS = {"incremental": ("k_sweep_pipe", "k_sweep_inc"), "full": ("k_sweep",)}


def stored_traffic(workload: str, precision: str, kernel: str = "k_eloc"):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE summary
    (profiles/<kernel>_<workload>_<precision>_hbm_traffic.md), or None when there is
    none for this workload or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{precision}_hbm_traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and line.split(":")[0] in ("traffic_bytes_per_launch", "source_sha256_16"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_sha256_16") != source_hash():
        return None
    return int(vals["traffic_bytes_per_launch"]) if "traffic_bytes_per_launch" in vals else None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="kagome432_L6F64")
    ap.add_argument("--precision", default="bf16", choices=["bf16", "bf16_1x", "fp32", "fp64"],
                    help="bf16: split (hi + lo) BF16 activations, BF16 weights; bf16_1x: single-pass BF16")
    ap.add_argument("--eloc-mode", default="incremental", choices=["incremental", "full"],
                    help="how the timed step evaluates the exchanged configurations")
    ap.add_argument("--compare", default="bf16_1x,fp32,fp64", help="other precisions timed on E_loc alone")
    ap.add_argument("--full-batch", type=int, default=512,
                    help="batch of the full-recompute local energy (context beside the incremental one)")
    ap.add_argument("--eloc-reps", type=int, default=3)
    ap.add_argument("--profile-steps", type=int, default=3, help="profiled steps after the timed ones")
    ap.add_argument("--cpu-samples", type=int, default=64)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline steps only (for profilers)")
    ap.add_argument("--no-graph", action="store_true", help="skip the HIP-graph replay timing")
    ap.add_argument("--no-tune", action="store_true", help="keep the default incremental shape")
    ap.add_argument("--shape", default=None, metavar="J,W,X",
                    help="pin the incremental local-energy kernel's shape (jobs in flight, waves, "
                         "samples per XCD) instead of tuning")
    ap.add_argument("--sweep-shape", default=None, metavar="J,W",
                    help="pin the incremental sweep kernel's shape (jobs in flight, waves)")
    ap.add_argument("--graph-reps", type=int, default=20, help="timed graph replays per component")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="also run a plain device copy of this many MiB (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as w
    from paper_2011_12453_amd import GNA

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    p = w.preset(args.workload)
    n, e = p.build_graph()
    F, L, B = p.n_features, p.n_layers, p.batch
    theta_np = w.glorot_theta(F, L, True, seed=p.theta_seed)
    spins_np = w.random_sz0_spins(B, n, p.spin_seed)
    fpe = flops_per_eval(n, len(e), F, L)
    bfl = ball_flops(n, e, F, L)                       # per bond, incremental evaluation
    acc_bytes = 8 if args.precision == "fp64" else 4
    brd, bwr = ball_bytes(n, e, F, L, acc_bytes)      # per bond, sampler proposal

    def anti_of(spins_now):
        return spins_now[:, e[:, 0]] != spins_now[:, e[:, 1]]

    def kernel_flops(mode, spins_now):
        a = anti_of(spins_now)
        return float((a * bfl[None, :]).sum()) if mode == "incremental" else float(a.sum()) * fpe
    log = lambda *a: print(*a, file=sys.stderr, flush=True)

    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy calibration: 3 copies of {nbytes} bytes")
        del src, dst

    # ---------------- headline: whole step ----------------
    g = GNA(n, e, F, L, tied=True, precision=args.precision, max_batch=B, device=dev, eloc_mode=args.eloc_mode)
    theta = torch.from_numpy(theta_np).to(dev)
    spins = torch.from_numpy(spins_np).to(dev)
    lp = torch.empty((B, 2), dtype=torch.float64, device=dev)
    # SGD on the energy per site with step 1e-3 (Section 3's update on E/N): the
    # total energy's gradient is extensive, and a step of 1e-3 on it freezes the
    # chains within a dozen steps (acceptance 0), a regime no VMC run stays in
    alpha = 1e-3 / n
    seed = 20201124
    counter = torch.zeros(1, dtype=torch.int64, device=dev)   # sampler's Philox counter base
    grad_buf = torch.empty(g.num_params, dtype=torch.float64, device=dev)
    el_buf = torch.empty((B, 2), dtype=torch.float64, device=dev)
    acc_buf = torch.empty(B, dtype=torch.int32, device=dev)

    theta_init, spins_init = theta.clone(), spins.clone()

    def step(stats=None):
        # gna_step: log psi, one sweep (counter advanced on the device), ISGO gradient, SGD
        stats = torch.empty(8, dtype=torch.float64, device=dev) if stats is None else stats
        g.step(theta, spins, lp, 1, seed, counter, alpha, grad=grad_buf, stats=stats, eloc=el_buf,
               n_accept=acc_buf)
        return stats

    tuned = None
    if args.shape or args.sweep_shape:
        if args.shape:
            j, wv, x = (int(v) for v in args.shape.split(","))
            g.set_shape(j, wv, x, which="eloc")
        if args.sweep_shape:
            j, wv = (int(v) for v in args.sweep_shape.split(","))
            g.set_shape(j, wv, 1, which="sweep")
        log(f"[bench] pinned shape: {g.config_info()}")
    elif args.eloc_mode == "incremental" and not args.no_tune:
        # the tuner times the incremental kernels' shapes on this batch (before any timing)
        tuned = g.autotune(theta, spins)
        log(f"[bench] autotune: {tuned}")
    shape = g.config_info()
    log(f"[bench] {p.name}: N={n} |E|={len(e)} F={F} L={L} B={B} {args.precision}; warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats_list, acc_list = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats_list.append(step())
        acc_list.append(acc_buf.sum())      # accepted swaps of the step's sweep (device scalar)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats_all = torch.stack(stats_list).cpu().numpy()
    acc_steps = torch.stack(acc_list).cpu().numpy().astype(np.float64) / (B * n)
    evals = float(stats_all[:, 6].sum())
    elapsed = t1 - t0
    value = evals / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s; {evals:.0f} E_loc evals; {value:.4g} evals/s; "
        f"acceptance per proposal {acc_steps.mean():.4f}")

    # per-kernel durations: a separate profiled pass of the same step (events on the
    # library's stream), continuing the trajectory
    spins_before = spins.cpu().numpy()
    g.profile_read()
    g.profile_enable(True)
    acc_prof = []
    for _ in range(args.profile_steps):
        step()
        acc_prof.append(acc_buf.sum())
    prof = g.profile_read()
    g.profile_enable(False)
    spins_after = spins.cpu().numpy()
    acc_prof = torch.stack(acc_prof).cpu().numpy().astype(np.float64)
    log("[bench] kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f}ms x{v[0]}" for k, v in sorted(prof.items())))

    # dominant kernel: algorithmic FLOPs per launch / mean launch time; the step's
    # local energy runs on the configurations its sweep left (spins_after per step
    # stands in for the profiled steps: the sweep moves chains but keeps bond statistics)
    kname = kernel_of(prof, ELOC_KERNELS[args.eloc_mode])
    kl, kms = prof.get(kname, (0, 0.0))
    eloc_ms = kms / max(kl, 1)
    kflops = kernel_flops(args.eloc_mode, spins_after)
    achieved = kflops / (eloc_ms * 1e-3) if kl else 0.0
    n_exch = float(anti_of(spins_after).sum())
    roofline = {"bound": "mfma", "kernel": kname, "achieved": achieved / 1e12,
                "peak": PEAK[args.precision] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[args.precision],
                "traffic": stored_traffic(p.name, args.precision, kname),
                "launch_ms": eloc_ms, "exchanges_per_launch": n_exch,
                "flops_per_exchange": kflops / max(n_exch, 1.0)}
    # the sampler: algorithmic bytes of its proposals (read for every anti-aligned
    # proposal, written for every accepted one) against the HBM peak
    roofline_sweep = None
    sname = kernel_of(prof, SWEEP_KERNELS[args.eloc_mode])
    sl, sms = prof.get(sname, (0, 0.0))
    if sl and args.eloc_mode == "incremental":
        a_frac = anti_of(np.concatenate([spins_before, spins_after])).mean(axis=0)   # per bond
        w_b = a_frac / max(a_frac.sum(), 1e-30)
        n_prop_anti = B * n * float(a_frac.mean())           # proposals drawn on anti-aligned bonds
        n_acc = float(acc_prof.mean())
        byt = n_prop_anti * float((w_b * brd).sum()) + n_acc * float((w_b * bwr).sum())
        s_ms = sms / sl
        roofline_sweep = {"bound": "hbm", "kernel": sname, "achieved": byt / (s_ms * 1e-3) / 1e9,
                          "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": byt / (s_ms * 1e-3) / HBM_PEAK,
                          "traffic": stored_traffic(p.name, args.precision, sname),
                          "launch_ms": s_ms, "algorithmic_bytes": byt,
                          "anti_aligned_proposals": n_prop_anti, "accepted": n_acc}

    # ---------------- the same step replayed from a captured HIP graph ----------------
    graph_info = None
    if not args.no_graph and not args.quick:
        # replay the same trajectory as the eager run: initial state, warm-up steps, timed steps
        stats_g = torch.empty(8, dtype=torch.float64, device=dev)
        theta.copy_(theta_init)
        spins.copy_(spins_init)
        counter.zero_()
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            g.set_stream(torch.cuda.current_stream())
            step(stats=stats_g)
        g.set_stream(torch.cuda.current_stream())
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        for _ in range(args.steps):
            graph.replay()
        torch.cuda.synchronize()
        tg1 = time.perf_counter()
        gms = 1e3 * (tg1 - tg0) / args.steps
        graph_info = {"ms_per_step": gms, "evals_per_s": (evals / args.steps) / (gms * 1e-3),
                      "note": "whole step captured once and replayed from the same initial state as the "
                              "eager run (same trajectory); evals per step from the timed eager steps"}
        log(f"[bench] graph replay: {gms:.2f} ms/step, {graph_info['evals_per_s']:.4g} evals/s")
        del graph

    # ---------------- E_loc alone: every precision at the same batch ----------------
    # incremental (the metric's evaluation): eager calls with per-kernel events, then
    # the call captured in a HIP graph (3 warm-up and `--graph-reps` timed replays,
    # median and min); full recompute at --full-batch as context (eager only)
    def graph_times(fn, reps):
        torch.cuda.synchronize()
        gr = torch.cuda.CUDAGraph()
        with torch.cuda.graph(gr):
            fn(torch.cuda.current_stream())
        for _ in range(3):
            gr.replay()
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in ev:
            a.record()
            gr.replay()
            b.record()
        torch.cuda.synchronize()
        ms = sorted(a.elapsed_time(b) for a, b in ev)
        del gr
        return ms[len(ms) // 2], ms[0]

    per_prec = {}
    eloc_out = {}
    other = "full" if args.eloc_mode == "incremental" else "incremental"
    runs = [(args.precision, args.eloc_mode), (args.precision, other)]
    runs += [(q, m) for q in args.compare.split(",") if q and q != args.precision for m in ("incremental", "full")]
    for prec, mode in runs:
        if args.quick and (prec, mode) != (args.precision, args.eloc_mode):
            continue
        Bp = B if mode == "incremental" else min(B, args.full_batch)
        gp = g if (prec, mode) == (args.precision, args.eloc_mode) else \
            GNA(n, e, F, L, tied=True, precision=prec, max_batch=Bp, device=dev, eloc_mode=mode)
        th0 = torch.from_numpy(theta_np).to(dev)
        sp0 = torch.from_numpy(spins_np[:Bp]).to(dev)
        if gp is not g and mode == "incremental" and not args.no_tune:
            log(f"[bench] autotune {prec}: {gp.autotune(th0, sp0)}")   # each precision in its own best shape
        el, nev = gp.local_energy(th0, sp0)        # warm
        torch.cuda.synchronize()
        reps = args.eloc_reps if mode == "incremental" else 1
        gp.profile_read()
        gp.profile_enable(True)
        ta = time.perf_counter()
        for _ in range(reps):
            el, nev = gp.local_energy(th0, sp0)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        pr = gp.profile_read()
        gp.profile_enable(False)
        ne = int(nev.item())
        rate = ne * reps / (tb - ta)
        kn = kernel_of(pr, ELOC_KERNELS[mode])
        kl2, kms2 = pr.get(kn, (1, 0.0))
        kf = kernel_flops(mode, spins_np[:Bp])
        key = f"{prec}_{mode}"
        per_prec[key] = {"evals_per_s": rate, "batch": Bp, "evals_per_call": ne,
                         "kernel": kn, "kernel_ms": kms2 / max(kl2, 1),
                         "kernel_tflops": kf / (kms2 / max(kl2, 1) * 1e-3) / 1e12,
                         "mfma_frac": kf / (kms2 / max(kl2, 1) * 1e-3) / PEAK[prec],
                         "note": "profiled eager calls (per-kernel events on)"}
        if not args.no_graph and not args.quick and mode == "incremental":
            el_g = torch.empty((Bp, 2), dtype=torch.float64, device=dev)
            nev_g = torch.empty(1, dtype=torch.int64, device=dev)

            def call(stream, gp=gp, th0=th0, sp0=sp0, el_g=el_g, nev_g=nev_g):
                gp.set_stream(stream)
                gp.local_energy(th0, sp0, out=el_g, n_evals=nev_g)
            med, mn = graph_times(call, args.graph_reps)
            gp.set_stream(torch.cuda.current_stream())
            per_prec[key].update({"graph_ms_median": med, "graph_ms_min": mn,
                                  "graph_evals_per_s": ne / (med * 1e-3)})
            log(f"[bench] E_loc {prec} {mode}: graph replay median {med:.2f} ms (min {mn:.2f}), "
                f"{ne / (med * 1e-3):.4g} evals/s")
        eloc_out[key] = el.cpu().numpy()
        log(f"[bench] E_loc {prec} {mode}: B={Bp} {rate:.4g} evals/s, {kn} {kms2 / max(kl2, 1):.2f} ms")
        if gp is not g:
            gp.close()

    # ---------------- sampler (a6) and reverse pass (a8) on their own ----------------
    components = None
    if not args.no_graph and not args.quick:
        th0 = torch.from_numpy(theta_np).to(dev)
        sp_c = torch.from_numpy(spins_np).to(dev)
        lp_c = g.logpsi(th0, sp_c)
        acc_c = torch.empty(B, dtype=torch.int32, device=dev)
        cot = torch.from_numpy(np.random.default_rng(0).normal(size=(B, 2))).to(dev)
        gr_c = torch.empty(g.num_params, dtype=torch.float64, device=dev)

        def sweep_call(stream):
            g.set_stream(stream)
            g.metropolis_sweep(th0, sp_c, lp_c, n_sweeps=1, seed=seed, counter_base=0, n_accept=acc_c)

        def vjp_call(stream):
            g.set_stream(stream)
            g.logpsi_vjp(th0, sp_c, cot, out=gr_c)
        sw_med, sw_min = graph_times(sweep_call, args.graph_reps)
        vj_med, vj_min = graph_times(vjp_call, args.graph_reps)
        g.set_stream(torch.cuda.current_stream())
        components = {"sweep_ms_median": sw_med, "sweep_ms_min": sw_min,
                      "sweep_proposals_per_s": B * n / (sw_med * 1e-3),
                      "sweep_acceptance_per_proposal": float(acc_c.sum().item()) / (B * n),
                      "vjp_ms_median": vj_med, "vjp_ms_min": vj_min,
                      "vjp_samples_per_s": B / (vj_med * 1e-3),
                      "note": "Glorot parameters and the initial batch (the step's trajectory moves both)"}
        log(f"[bench] sweep (1 sweep, {B} chains): {sw_med:.2f} ms; VJP ({B} samples): {vj_med:.2f} ms")

    # ---------------- CPU baseline (FP64 oracle) and error columns ----------------
    cpu = None
    if not args.no_cpu_baseline and not args.quick:
        import oracle
        try:
            from threadpoolctl import threadpool_info
            threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        S = min(args.cpu_samples, B)
        sub = spins_np[:S]
        tc = time.perf_counter()
        ref = oracle.local_energy(theta_np, sub, n, e, F, L)
        tcpu = time.perf_counter() - tc
        ne_cpu = oracle.n_evals(sub, e)
        cpu = {"value": ne_cpu / tcpu, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"first {S} of {B} configurations ({ne_cpu} log-psi evals, {tcpu:.1f}s)"}
        off_ref = ref - len(e) / 4.0          # the part a constant psi gets wrong
        for prec, el in eloc_out.items():
            got = el[:S, 0] + 1j * el[:S, 1]
            es, rs = got.real.mean() / n, ref.real.mean() / n
            off_rel = np.abs(got - ref) / np.abs(off_ref)           # per row
            off_big = np.abs(got - ref) / np.max(np.abs(off_ref))   # over the largest part
            per_prec[prec].update({
                "err_energy_per_site": abs(es - rs) / max(abs(rs), 1e-2),
                "err_offdiag_rel_median": float(np.median(off_rel)),
                "err_offdiag_max_over_largest_part": float(off_big.max()),
                "err_offdiag_mean_rel": float(abs(np.mean(got - len(e) / 4.0) - np.mean(off_ref)) /
                                              abs(np.mean(off_ref))),
                "err_eloc_max_rel": float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))),
                "bound_energy_per_site": BOUND[prec.rsplit("_", 1)[0]],
                "error_sample": S})
        log(f"[bench] oracle: {cpu['value']:.4g} evals/s on {threads} threads")

    kind = p.graph.split(":")[0]
    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if args.precision.startswith("bf16") else args.precision, "data": "synthetic",
        "config": {"workload": p.name, "lattice": LATTICE.get(kind, kind), "graph": p.graph, "sites": n,
                   "bonds": len(e), "layers": L, "features": F, "tied": True, "batch": B,
                   "precision": args.precision,
                   "step": "gna_step: logpsi + 1 Metropolis sweep + ISGO update (logpsi, E_loc, stats, VJP) + SGD",
                   "eloc_mode": args.eloc_mode,
                   "shape": shape,
                   "evals_per_step": evals / args.steps,
                   "sgd_step": alpha,
                   "acceptance_per_proposal": float(acc_steps.mean()),
                   "acceptance_per_step": [float(a) for a in acc_steps]},
        "roofline": roofline,
        "roofline_sweep": roofline_sweep,
        "cpu_baseline": cpu,
        "graph": graph_info,
        "components": components,
        "precisions": per_prec,
        "kernels_ms_per_step": {k: v[1] / args.profile_steps for k, v in sorted(prof.items())},
    }
    head = per_prec.get(f"{args.precision}_{args.eloc_mode}", {})
    if "err_energy_per_site" in head:   # the stated error bound of the headline precision
        bound = BOUND[args.precision]
        out["accuracy"] = {"precision": args.precision, "err_energy_per_site": head["err_energy_per_site"],
                           "bound": bound, "within_bound": bool(head["err_energy_per_site"] < bound),
                           "err_offdiag_rel_median": head["err_offdiag_rel_median"],
                           "err_offdiag_max_over_largest_part": head["err_offdiag_max_over_largest_part"],
                           "sample": cpu["sample"]}
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
