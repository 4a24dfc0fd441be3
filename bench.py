#!/usr/bin/env python
"""Benchmark: log-psi evaluations per second inside the local energy, 432-site Kagome.

One step is one pass of the whole hot path over a batch of 2048 chains on the
12x12x3 Kagome torus (864 bonds, GCN with 6 tied layers of width 64):

    refresh log psi -> one Metropolis sweep (432 proposals per chain) ->
    ISGO update (log psi, E_loc over every exchanged configuration, weights,
    reverse pass) -> SGD update

``value`` = local-energy log-psi evaluations (the library's exact count) per
second of whole-step wall time, BF16 layer products (single-pass BF16 operands by
default; the split-activation BF16, FP32 and FP64 modes are timed on the local
energy alone beside it, each with its error against the oracle).  Per-kernel
durations come from HIP events the library records on its stream; the roofline
entry is for the dominant kernel.  The CPU baseline times the FP64 oracle on a
bounded prefix of the same batch, and its outputs give the error columns.
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


def flops_per_eval(n, n_edges, F, L):
    """Algorithmic FLOPs of one log-psi evaluation: per layer the [M|H] W product
    (2 N 2F F) and the aggregation (2 per stored adjacency entry per feature), plus
    the two-head readout.  tanh is not counted."""
    return L * (2 * n * 2 * F * F + 2 * (2 * n_edges) * F) + 2 * 2 * n * F


def ball_flops(n, edges, F, L):
    """Algorithmic FLOPs of one incremental evaluation for each bond: at layer l the
    message product of the ball C_{l-1} and the self product, aggregation and
    activation input of the ball C_l (C_0 = the bond, C_l = C_{l-1} plus neighbours),
    plus the two-head readout difference over C_L."""
    import numpy as np
    adj = [[] for _ in range(n)]
    for a, b in edges:
        adj[a].append(b)
        adj[b].append(a)
    deg = np.array([len(x) for x in adj])
    out = []
    for a, b in edges:
        balls = [{int(a), int(b)}]
        for _ in range(L):
            nxt = set(balls[-1])
            for u in balls[-1]:
                nxt.update(adj[u])
            balls.append(nxt)
        f = 0
        for l in range(1, L + 1):
            f += 2 * len(balls[l - 1]) * F * F + 2 * len(balls[l]) * F * F
            f += 2 * int(deg[list(balls[l])].sum()) * F
        f += 2 * 2 * len(balls[L]) * F
        out.append(f)
    return np.array(out, dtype=np.float64)


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


def stored_traffic(workload: str, precision: str, kernel: str = "k_eloc"):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE summary,
    or None when there is none for this workload or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload.split('_')[0]}_{precision}_hbm_traffic.md")
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
    ap.add_argument("--precision", default="bf16_1x", choices=["bf16", "bf16_1x", "fp32", "fp64"],
                    help="bf16_1x: single-pass BF16 operands; bf16: split (hi + lo) BF16 activations")
    ap.add_argument("--eloc-mode", default="incremental", choices=["incremental", "full"],
                    help="how the timed step evaluates the exchanged configurations")
    ap.add_argument("--compare", default="bf16,fp32,fp64", help="other precisions timed on E_loc alone")
    ap.add_argument("--compare-batch", type=int, default=512)
    ap.add_argument("--eloc-reps", type=int, default=3)
    ap.add_argument("--cpu-samples", type=int, default=8)
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
    anti = (spins_np[:, e[:, 0]] != spins_np[:, e[:, 1]])
    inc_flops_batch = float((anti * bfl[None, :]).sum())   # initial batch; the step's spins drift

    def kernel_flops(mode, spins_now):
        a = (spins_now[:, e[:, 0]] != spins_now[:, e[:, 1]])
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
    alpha = 1e-3
    seed = 20201124
    counter = torch.zeros(1, dtype=torch.int64, device=dev)   # sampler's Philox counter base
    grad_buf = torch.empty(g.num_params, dtype=torch.float64, device=dev)
    el_buf = torch.empty((B, 2), dtype=torch.float64, device=dev)
    acc_buf = torch.empty(B, dtype=torch.int32, device=dev)

    theta_init, spins_init = theta.clone(), spins.clone()

    def step(k, stats=None):
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
    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    g.profile_read()                 # discard
    g.profile_enable(True)
    stats_list = []
    kflops = 0.0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        stats_list.append(step(args.warmup + k))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # algorithmic work of the local-energy kernel: recompute from the final spins of
    # each step would need copies inside the timed loop; the step's sweep changes the
    # configurations but not their bond statistics, so the final batch stands in
    kflops = kernel_flops(args.eloc_mode, spins.cpu().numpy()) * args.steps
    prof = g.profile_read()
    g.profile_enable(False)
    stats_all = torch.stack(stats_list).cpu().numpy()
    evals = float(stats_all[:, 6].sum())
    elapsed = t1 - t0
    value = evals / elapsed
    log(f"[bench] {args.steps} steps in {elapsed:.3f}s; {evals:.0f} E_loc evals; {value:.4g} evals/s")
    log("[bench] kernels: " + ", ".join(f"{k} {v[1] / max(v[0], 1):.3f}ms x{v[0]}" for k, v in sorted(prof.items())))

    # dominant kernel: algorithmic FLOPs per launch / mean launch time
    kname = "k_eloc_inc" if args.eloc_mode == "incremental" else "k_eloc"
    kl, kms = prof.get(kname, (0, 0.0))
    eloc_ms = kms / max(kl, 1)
    achieved = (kflops / max(kl, 1)) / (eloc_ms * 1e-3) if kl else 0.0
    roofline = {"bound": "mfma", "kernel": kname, "achieved": achieved / 1e12,
                "peak": PEAK[args.precision] / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK[args.precision],
                "traffic": stored_traffic(p.name, args.precision, kname),
                "launch_ms": eloc_ms,
                "flops_per_eval": (kflops / args.steps) / max(1.0, evals / args.steps - B)}

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
            step(0, stats=stats_g)
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

    # ---------------- E_loc alone: both modes, every precision ----------------
    # one eager call with per-kernel events (kernel time for the roofline), then the call
    # captured in a HIP graph: 3 warm-up and `--graph-reps` timed replays, median and min
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
    runs = [(args.precision, args.eloc_mode), (args.precision, "full" if args.eloc_mode == "incremental" else "incremental")]
    runs += [(q, m) for q in args.compare.split(",") if q and q != args.precision for m in ("incremental", "full")]
    for prec, mode in runs:
        if args.quick and (prec, mode) != (args.precision, args.eloc_mode):
            continue
        Bp = B if prec == args.precision else min(B, args.compare_batch)
        gp = g if (prec, mode) == (args.precision, args.eloc_mode) else \
            GNA(n, e, F, L, tied=True, precision=prec, max_batch=Bp, device=dev, eloc_mode=mode)
        th0 = torch.from_numpy(theta_np).to(dev)
        sp0 = torch.from_numpy(spins_np[:Bp]).to(dev)
        if gp is not g and mode == "incremental" and not args.no_tune:
            log(f"[bench] autotune {prec}: {gp.autotune(th0, sp0)}")   # each precision in its own best shape
        el, nev = gp.local_energy(th0, sp0)        # warm
        torch.cuda.synchronize()
        gp.profile_read()
        gp.profile_enable(True)
        ta = time.perf_counter()
        for _ in range(args.eloc_reps):
            el, nev = gp.local_energy(th0, sp0)
        torch.cuda.synchronize()
        tb = time.perf_counter()
        pr = gp.profile_read()
        gp.profile_enable(False)
        ne = int(nev.item())
        rate = ne * args.eloc_reps / (tb - ta)
        kn = "k_eloc_inc" if mode == "incremental" else "k_eloc"
        kl2, kms2 = pr.get(kn, (1, 0.0))
        kf = kernel_flops(mode, spins_np[:Bp])
        key = f"{prec}_{mode}"
        per_prec[key] = {"evals_per_s": rate, "batch": Bp, "evals_per_call": ne,
                         "kernel": kn, "kernel_ms": kms2 / max(kl2, 1),
                         "kernel_tflops": kf / (kms2 / max(kl2, 1) * 1e-3) / 1e12,
                         "mfma_frac": kf / (kms2 / max(kl2, 1) * 1e-3) / PEAK[prec]}
        if not args.no_graph and not args.quick:
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
                      "vjp_ms_median": vj_med, "vjp_ms_min": vj_min,
                      "vjp_samples_per_s": B / (vj_med * 1e-3)}
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
        S = args.cpu_samples
        sub = spins_np[:S]
        tc = time.perf_counter()
        ref = oracle.local_energy(theta_np, sub, n, e, F, L)
        tcpu = time.perf_counter() - tc
        ne_cpu = oracle.n_evals(sub, e)
        cpu = {"value": ne_cpu / tcpu, "unit": "evals/s", "cores": threads, "kind": "oracle",
               "sample": f"first {S} of {B} configurations ({ne_cpu} log-psi evals, {tcpu:.1f}s)"}
        try:   # the same oracle on one thread, on a smaller sample
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1):
                S1 = max(1, S // 4)
                t1c = time.perf_counter()
                oracle.local_energy(theta_np, spins_np[:S1], n, e, F, L)
                t1c = time.perf_counter() - t1c
            cpu["value_1_thread"] = oracle.n_evals(spins_np[:S1], e) / t1c
            cpu["sample_1_thread"] = f"first {S1} configurations, {t1c:.1f}s"
        except Exception as exc:   # threadpoolctl missing: the all-core figure stands alone
            cpu["value_1_thread"] = None
            cpu["sample_1_thread"] = f"not measured ({type(exc).__name__})"
        for prec, el in eloc_out.items():
            got = el[:S]
            es, rs = got[:, 0].mean() / n, ref.real.mean() / n
            per_prec[prec]["err_energy_per_site"] = abs(es - rs) / max(abs(rs), 1e-2)
            per_prec[prec]["err_eloc_max_rel"] = float(np.max(np.abs(got[:, 0] - ref.real) +
                                                              np.abs(got[:, 1] - ref.imag)) / np.max(np.abs(ref)))
        log(f"[bench] oracle: {cpu['value']:.4g} evals/s on {threads} threads")

    out = {
        "metric": METRIC, "value": value, "unit": "evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16" if args.precision.startswith("bf16") else args.precision, "data": "synthetic",
        "config": {"workload": p.name, "lattice": "12x12x3 kagome torus", "sites": n, "bonds": len(e),
                   "layers": L, "features": F, "tied": True, "batch": B,
                   "step": "gna_step: logpsi + 1 Metropolis sweep + ISGO update (logpsi, E_loc, stats, VJP) + SGD",
                   "eloc_mode": args.eloc_mode,
                   "shape": shape,
                   "evals_per_step": evals / args.steps},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "graph": graph_info,
        "components": components,
        "precisions": per_prec,
        "kernels_ms_per_step": {k: v[1] / args.steps for k, v in sorted(prof.items())},
    }
    head = per_prec.get(f"{args.precision}_{args.eloc_mode}", {})
    if "err_energy_per_site" in head:   # the stated error bound of the headline precision
        bound = {"fp64": 1e-10, "fp32": 1e-5}.get(args.precision, 1e-3)
        out["accuracy"] = {"precision": args.precision, "err_energy_per_site": head["err_energy_per_site"],
                           "bound": bound, "within_bound": bool(head["err_energy_per_site"] < bound),
                           "sample": cpu["sample"]}
    print(json.dumps(out))
    g.close()


if __name__ == "__main__":
    main()
