"""Grouping of duplicated states on the GPU (Section 3) against the oracle: the
distinct rows, their order of first occurrence and their counts are integer work and
must match exactly; the ISGO estimates over the grouped batch must equal those over
the full batch."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _ctx(n, e, max_batch, F=16, L=2, prec="fp64"):
    from paper_2011_12453_amd import GNA
    print(f"[gpu] group ctx N={n} B<={max_batch} {prec}", file=sys.stderr, flush=True)
    return GNA(n, e, F, L, tied=True, precision=prec, max_batch=max_batch, device=DEV)


def _dup_batch(B, n, seed, pool):
    rng = np.random.default_rng(seed)
    p = w.random_sz0_spins(pool, n, seed)
    return p[rng.integers(0, pool, size=B)]


def _check(g, s):
    u, c, nu = g.group_duplicates(torch.from_numpy(s).to(DEV))
    u, c, U = u.cpu().numpy(), c.cpu().numpy(), int(nu.item())
    ru, rc, _ = oracle.group_duplicates(s)
    print(f"[gpu] group B={len(s)} N={s.shape[1]}: {U} unique", file=sys.stderr, flush=True)
    assert U == len(ru)
    assert np.array_equal(u[:U], ru) and np.array_equal(c[:U], rc)
    if U < len(s):                        # padding rows: the first row, count 0
        assert np.all(u[U:] == u[0]) and np.all(c[U:] == 0.0)
    return U


@pytest.mark.parametrize("B,n,pool", [(1024, 12, 300), (2000, 108, 50), (777, 36, 777), (4096, 432, 4096)],
                         ids=["kagome12", "kagome108_heavy", "tri36_ragged", "kagome432_distinct"])
def test_group_matches_oracle(B, n, pool):
    s = _dup_batch(B, n, B + n, pool) if pool < B else w.random_sz0_spins(B, n, B + n)
    g = _ctx(n, w.kagome(2, 2)[1] if n == 12 else [(i, (i + 1) % n) for i in range(n)], B)
    U = _check(g, s)
    if pool >= B:
        assert U == B
    g.close()


def test_group_edge_cases():
    n, e = w.kagome(2, 2)
    g = _ctx(n, e, 64)
    # every Sz=0 state once: all distinct, in order
    st = oracle.exact.enumerate_sz0(n)[:64]
    assert _check(g, st) == 64
    # all rows equal; a single row; a batch of one repeated twice
    one = w.random_sz0_spins(1, n, 5)
    assert _check(g, np.repeat(one, 64, axis=0)) == 1
    assert _check(g, one) == 1
    assert _check(g, np.repeat(one, 2, axis=0)) == 1
    # empty batch: n_unique is written as 0
    u, c, nu = g.group_duplicates(torch.empty((0, n), dtype=torch.int8, device=DEV))
    assert int(nu.item()) == 0
    # the same context again on another batch (the table is cleared per call)
    assert _check(g, _dup_batch(64, n, 9, 10)) <= 10
    g.close()


def test_group_rejects_bad_arguments():
    from paper_2011_12453_amd.binding import GnaError
    n, e = w.kagome(2, 2)
    g = _ctx(n, e, 8)
    s = torch.from_numpy(w.random_sz0_spins(8, n, 1)).to(DEV)
    with pytest.raises(GnaError):
        g.group_duplicates(s, uniq=s)
    with pytest.raises(GnaError):
        g.group_duplicates(torch.from_numpy(w.random_sz0_spins(9, n, 1)).to(DEV))
    g.close()


@pytest.mark.parametrize("mode", ["full", "incremental"])
def test_isgo_on_grouped_batch_equals_full_batch(mode):
    from paper_2011_12453_amd import GNA
    n, e = w.kagome(2, 2)
    F, L, B = 16, 2, 1024
    th_old = w.glorot_theta(F, L, True, seed=6, weight_scale=1.5, bias_std=0.3)
    th_new = th_old + 0.03 * np.random.default_rng(1).normal(size=th_old.size)
    s = _dup_batch(B, n, 3, 200)
    g = GNA(n, e, F, L, tied=True, precision="fp64", max_batch=B, device=DEV, eloc_mode=mode)
    to = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(DEV)
    sp = to(s)
    lp_old = g.logpsi(to(th_old), sp)
    g_full, st_full, _ = g.isgo_grad(to(th_new), sp, lp_old)
    u, c, nu = g.group_duplicates(sp)
    U = int(nu.item())
    lp_u = g.logpsi(to(th_old), u[:U].contiguous())
    g_grp, st_grp, _ = g.isgo_grad(to(th_new), u[:U].contiguous(), lp_u, counts=c[:U].contiguous())
    # and the padded [B] output passed on unchanged (count-0 rows add nothing)
    lp_p = g.logpsi(to(th_old), u)
    g_pad, st_pad, _ = g.isgo_grad(to(th_new), u, lp_p, counts=c)
    g.close()
    g_full, g_grp, g_pad = (x.cpu().numpy() for x in (g_full, g_grp, g_pad))
    st_full, st_grp, st_pad = (x.cpu().numpy() for x in (st_full, st_grp, st_pad))
    print(f"[gpu] grouped isgo {mode}: {U} of {B} rows, evals {st_grp[6]:.0f} vs {st_full[6]:.0f}",
          file=sys.stderr, flush=True)
    assert U < B and st_grp[6] < st_full[6]
    for gg, ss in ((g_grp, st_grp), (g_pad, st_pad)):
        assert abs(ss[0] - st_full[0]) < 1e-12 * abs(st_full[0])
        assert abs(ss[2] - st_full[2]) < 1e-11 * st_full[2]
        assert np.max(np.abs(gg - g_full)) < 1e-11 * np.max(np.abs(g_full))


def test_group_graph_replay():
    # the grouping clears its table with fill kernels (no memset), so it can be captured
    # and replayed: each replay on new rows copied into the captured input
    n, e = w.kagome(2, 2)
    B = 512
    g = _ctx(n, e, B)
    sp = torch.from_numpy(_dup_batch(B, n, 1, 100)).to(DEV)
    u = torch.empty((B, n), dtype=torch.int8, device=DEV)
    c = torch.empty(B, dtype=torch.float64, device=DEV)
    nu = torch.empty(1, dtype=torch.int32, device=DEV)
    g.group_duplicates(sp, u, c, nu)             # eager once before capture
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        g.set_stream(torch.cuda.current_stream())
        g.group_duplicates(sp, u, c, nu)
    g.set_stream(torch.cuda.current_stream())
    for k in range(3):
        s_new = _dup_batch(B, n, 10 + k, 50 + 100 * k)
        sp.copy_(torch.from_numpy(s_new).to(DEV))
        graph.replay()
        torch.cuda.synchronize()
        ru, rc, _ = oracle.group_duplicates(s_new)
        U = int(nu.item())
        assert U == len(ru) and np.array_equal(u[:U].cpu().numpy(), ru) and np.array_equal(c[:U].cpu().numpy(), rc)
        g.group_duplicates(torch.from_numpy(s_new[::-1].copy()).to(DEV))   # eager work between replays
        torch.cuda.synchronize()
    g.close()
