"""The sampling-iteration loop of Section 3 on top of the library's entry points.

Each iteration draws fresh Metropolis samples, optionally groups duplicated states
into unique states with counts, then takes several ISGO parameter updates on those
same samples (Eq. 3): the weights compare the wavefunction being optimised with the
one the samples were drawn from, and the loop leaves an iteration early once the
effective sample size of the weights falls below a fraction of its value at the
first update (the reweighting has drifted too far).  A checkpoint (parameters,
chains, sampler counter, iteration) can be written after every iteration and the
loop resumed from it; parameters trained on one graph can start another graph's
optimisation (Section 4.2: a 12-site ansatz reused on 432 sites), because the
parameters of Eq. 1 do not depend on the number of sites.  All arithmetic runs in
the library's kernels; this module only sequences the calls and reads the
statistics back.
"""
from __future__ import annotations

import numpy as np
import torch

from .binding import GNA, STAT_FIELDS

_CKPT_KEYS = ("theta", "spins", "counter", "iteration", "n_features", "n_layers", "tied", "activation")


def isgo_vmc(g: GNA, theta: torch.Tensor, spins: torch.Tensor, n_iters: int, n_updates: int,
             lr: float, n_sweeps: int = 1, burn_in: int = 10, seed: int = 0, ess_min: float = 0.5,
             counter_base: int = 0, group: bool = False, start_iter: int = 0,
             checkpoint: str | None = None):
    """Optimise ``theta`` in place; ``spins`` [B, N] are the chains (advanced in place).

    ``group``: run the updates on the unique states with counts (the estimates are
    those of the full batch; fewer local energies are evaluated).  ``checkpoint``:
    path written after every iteration (see ``save_checkpoint``); resume with
    ``start_iter`` and ``counter_base`` from it and ``burn_in=0``.

    Returns a list of per-update dicts (iteration, update, energy per site, its
    imaginary part, variance, ESS, rows evaluated) and the next counter base of the
    sampler.
    """
    B, N = spins.shape
    ess_i = STAT_FIELDS.index("ess")
    lp = g.logpsi(theta, spins)
    cb = counter_base
    if burn_in:
        g.metropolis_sweep(theta, spins, lp, n_sweeps=burn_in, seed=seed, counter_base=cb)
        cb += burn_in * N
    history = []
    for it in range(start_iter, start_iter + n_iters):
        g.metropolis_sweep(theta, spins, lp, n_sweeps=n_sweeps, seed=seed, counter_base=cb)
        cb += n_sweeps * N
        if group:
            uniq, counts, n_unique = g.group_duplicates(spins)
            U = int(n_unique.item())
            samples, counts = uniq[:U].contiguous(), counts[:U].contiguous()
            lp_old = g.logpsi(theta, samples)
        else:
            samples, counts, lp_old = spins, None, lp.clone()   # the distribution the samples come from
        ess0 = None
        for k in range(n_updates):
            grad, stats, _ = g.isgo_grad(theta, samples, lp_old, counts=counts)
            st = stats.cpu().numpy()
            if ess0 is None:
                ess0 = st[ess_i]
            elif st[ess_i] < ess_min * ess0:
                break
            history.append({"iteration": it, "update": k, "energy_per_site": st[0] / N,
                            "energy_imag": st[1], "variance": st[2], "ess": st[ess_i],
                            "rows": int(samples.shape[0])})
            g.sgd_update(theta, grad, lr)
        lp = g.logpsi(theta, spins)
        if checkpoint:
            save_checkpoint(checkpoint, g, theta, spins, cb, it + 1)
    return history, cb


def save_checkpoint(path: str, g: GNA, theta: torch.Tensor, spins: torch.Tensor, counter: int,
                    iteration: int) -> None:
    """Parameters, chains, sampler counter and next iteration, as a NumPy archive
    (no pickled objects)."""
    np.savez(path, theta=theta.detach().cpu().numpy(), spins=spins.detach().cpu().numpy(),
             counter=np.uint64(counter), iteration=np.int64(iteration),
             n_features=np.int64(g.n_features), n_layers=np.int64(g.n_layers), tied=np.int64(g.tied),
             activation=np.int64(g.activation))


def load_checkpoint(path: str, g: GNA) -> dict:
    """Read a checkpoint for context ``g`` (same F, L, weight sharing and activation;
    the chains must have g's number of sites).  Returns theta and spins on g's
    device, the counter and the next iteration."""
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in _CKPT_KEYS}
    for k, v in (("n_features", g.n_features), ("n_layers", g.n_layers), ("tied", int(g.tied)),
                 ("activation", g.activation)):
        if int(d[k]) != int(v):
            raise ValueError(f"checkpoint {k} = {int(d[k])}, context has {v}")
    if d["spins"].shape[1] != g.n_sites:
        raise ValueError(f"checkpoint chains have {d['spins'].shape[1]} sites, context has {g.n_sites}")
    return {"theta": torch.from_numpy(d["theta"]).to(g.device), "spins": torch.from_numpy(d["spins"]).to(g.device),
            "counter": int(d["counter"]), "iteration": int(d["iteration"])}


def transfer_theta(theta: torch.Tensor, src: GNA, dst: GNA) -> torch.Tensor:
    """Parameters trained with context ``src`` as the starting point on ``dst``'s graph.
    Eq. 1's weights act per node and per edge, so they carry over unchanged between
    graphs of any size; only F, L, weight sharing and the activation must agree."""
    for k in ("n_features", "n_layers", "tied", "activation"):
        if getattr(src, k) != getattr(dst, k):
            raise ValueError(f"{k} differs: {getattr(src, k)} vs {getattr(dst, k)}")
    return theta.detach().to(dst.device, copy=True)
