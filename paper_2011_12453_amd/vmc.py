"""The sampling-iteration loop of Section 3 on top of the library's entry points.

Each iteration draws fresh Metropolis samples, then takes several ISGO parameter
updates on those same samples (Eq. 3): the weights compare the wavefunction being
optimised with the one the samples were drawn from, and the loop leaves an
iteration early once the effective sample size of the weights falls below a
fraction of the batch (the reweighting has drifted too far).  All arithmetic runs
in the library's kernels; this module only sequences the calls and reads the
statistics back.
"""
from __future__ import annotations

import torch

from .binding import GNA, STAT_FIELDS


def isgo_vmc(g: GNA, theta: torch.Tensor, spins: torch.Tensor, n_iters: int, n_updates: int,
             lr: float, n_sweeps: int = 1, burn_in: int = 10, seed: int = 0, ess_min: float = 0.5,
             counter_base: int = 0):
    """Optimise ``theta`` in place; ``spins`` [B, N] are the chains (advanced in place).

    Returns a list of per-update dicts (iteration, update, energy per site, its
    imaginary part, variance, ESS) and the next counter base of the sampler.
    """
    B, N = spins.shape
    ess_i = STAT_FIELDS.index("ess")
    lp = g.logpsi(theta, spins)
    cb = counter_base
    if burn_in:
        g.metropolis_sweep(theta, spins, lp, n_sweeps=burn_in, seed=seed, counter_base=cb)
        cb += burn_in * N
    history = []
    for it in range(n_iters):
        g.metropolis_sweep(theta, spins, lp, n_sweeps=n_sweeps, seed=seed, counter_base=cb)
        cb += n_sweeps * N
        lp_old = lp.clone()                    # the distribution the samples come from
        for k in range(n_updates):
            grad, stats, _ = g.isgo_grad(theta, spins, lp_old)
            st = stats.cpu().numpy()
            if k > 0 and st[ess_i] < ess_min * B:
                break
            history.append({"iteration": it, "update": k, "energy_per_site": st[0] / N,
                            "energy_imag": st[1], "variance": st[2], "ess": st[ess_i]})
            g.sgd_update(theta, grad, lr)
        lp = g.logpsi(theta, spins)
    return history, cb
