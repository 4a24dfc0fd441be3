"""gna_local_energy_noalloc (the local energy with the library's static scratch, for
callers that cannot allocate) through the C ABI: the same results as
gna_local_energy on two calls in a row, the second with a smaller batch, in both
evaluation modes and with the layer-pipelined kernel; a batch whose scratch exceeds the
static array is refused before anything is enqueued."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("mode,prec", [("full", "fp64"), ("incremental", "fp64"), ("incremental", "bf16")])
def test_noalloc_equals_local_energy_twice(mode, prec):
    from paper_2011_12453_amd import GNA
    n, e = w.kagome(6, 6)
    F, L = 32, 4
    theta = w.glorot_theta(F, L, True, seed=3, weight_scale=1.5, bias_std=0.3)
    spins = w.random_sz0_spins(96, n, 41)
    print(f"[gpu] noalloc ctx kagome108 {mode} {prec}", file=sys.stderr, flush=True)
    g = GNA(n, e, F, L, tied=True, precision=prec, max_batch=96, device=DEV, eloc_mode=mode)
    th = _dev(theta)
    for B in (96, 37):      # the second call smaller: stale scratch beyond B must not matter
        sp = _dev(spins[:B])
        ref, nref = g.local_energy(th, sp)
        out = torch.full((B, 2), float("nan"), dtype=torch.float64, device=DEV)
        nev = torch.full((1,), -7, dtype=torch.int64, device=DEV)
        g.local_energy_noalloc(th, sp, out, nev)
        torch.cuda.synchronize()
        print(f"[gpu] noalloc B={B}: max |diff| {torch.max(torch.abs(out - ref)).item():.2e}", file=sys.stderr,
              flush=True)
        assert torch.equal(out, ref)                     # same kernels, same order: identical
        assert int(nev.item()) == int(nref.item()) == oracle.n_evals(spins[:B], e)
        out2 = torch.empty((B, 2), dtype=torch.float64, device=DEV)
        g.local_energy_noalloc(th, sp, out2)             # counter in the static scratch
        torch.cuda.synchronize()
        assert torch.equal(out2, ref)
    if prec == "fp64":   # and the oracle on a few rows of the last call
        el = oracle.local_energy(theta, spins[:4], n, e, F, L)
        got = out2.cpu().numpy()[:4]
        assert np.max(np.abs(got[:, 0] - el.real) + np.abs(got[:, 1] - el.imag)) < 1e-11 * np.max(np.abs(el))
    g.close()


def test_noalloc_pipelined_equals_local_energy_twice():
    # the layer-pipelined local-energy kernel keeps its exchange terms in the static
    # scratch too
    from paper_2011_12453_amd import GNA
    n, e = w.kagome(6, 6)
    F, L = 32, 4
    theta = w.glorot_theta(F, L, True, seed=5, weight_scale=1.5, bias_std=0.3)
    spins = w.random_sz0_spins(96, n, 43)
    print("[gpu] noalloc ctx kagome108 incremental bf16 pipelined/16", file=sys.stderr, flush=True)
    g = GNA(n, e, F, L, tied=True, precision="bf16", max_batch=96, device=DEV, eloc_mode="incremental")
    g.set_shape(0, 16, 2)
    assert g.config_info()["jobs_in_flight"] == 0
    th = _dev(theta)
    for B in (96, 37):
        sp = _dev(spins[:B])
        ref, nref = g.local_energy(th, sp)
        out = torch.full((B, 2), float("nan"), dtype=torch.float64, device=DEV)
        nev = torch.full((1,), -7, dtype=torch.int64, device=DEV)
        g.local_energy_noalloc(th, sp, out, nev)
        torch.cuda.synchronize()
        print(f"[gpu] noalloc pipelined B={B}: max |diff| {torch.max(torch.abs(out - ref)).item():.2e}",
              file=sys.stderr, flush=True)
        assert torch.equal(out, ref)
        assert int(nev.item()) == int(nref.item()) == oracle.n_evals(spins[:B], e)
    g.close()


def test_noalloc_pipelined_refuses_terms_beyond_its_scratch():
    from paper_2011_12453_amd import GNA, GnaError
    n, e = w.kagome(6, 6)
    B = 20000                    # 216 bonds x 16 bytes of exchange terms per sample: above 64 MiB
    g = GNA(n, e, 32, 2, tied=True, precision="bf16", max_batch=B, device=DEV, eloc_mode="incremental",
            act_budget_bytes=1 << 20)
    g.set_shape(0, 16, 2)
    th = _dev(w.glorot_theta(32, 2, True, seed=1))
    sp = _dev(w.random_sz0_spins(B, n, 7))
    out = torch.zeros((B, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(GnaError, match="static scratch"):
        g.local_energy_noalloc(th, sp, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0          # nothing was enqueued
    g.close()


def test_noalloc_refuses_batches_beyond_its_scratch():
    from paper_2011_12453_amd import GNA, GnaError
    n, e = w.kagome(2, 2)
    B = 1 << 21                  # at least 52 bytes of scratch per sample: above the 64 MiB array
    g = GNA(n, e, 16, 2, tied=True, precision="fp64", max_batch=B, device=DEV, eloc_mode="full",
            act_budget_bytes=1 << 20)
    th = _dev(w.glorot_theta(16, 2, True, seed=1))
    sp = torch.ones((B, n), dtype=torch.int8, device=DEV)
    out = torch.zeros((B, 2), dtype=torch.float64, device=DEV)
    with pytest.raises(GnaError, match="static scratch"):
        g.local_energy_noalloc(th, sp, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0          # nothing was enqueued
    g.close()
