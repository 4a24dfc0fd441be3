"""FP64 oracle: graph neural ansatz, Heisenberg local energy, ISGO statistics and gradient.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.  Plain NumPy/SciPy in
float64 / complex128; every step follows the paper's definitions in their order,
with library matmuls as the only primitives.

Readings of the paper taken here (each one is listed with its reason in the
design notes of the repository):

* Eq. (1) with f = tanh; the one-hot occupation is embedded as
  ``H0 = tanh(onehot(x) W_e + b_e)`` (Section 2 says "nonlinearly transformed").
* ``[A_hat H ; H]`` puts the neighbour message first, the node's own row second.
* ``A_hat = D^-1/2 A D^-1/2`` without self-loops; a node of degree 0 has a zero row.
* Readout (Section 2): concatenate the last embedding with the one-hot input, sum
  over sites, then two one-unit dense heads give log|psi| and the phase (the
  two-head complex form named in Section 5).
* Local energy of the spin-1/2 Heisenberg model
  ``E(s) = sum_<ij> [Jz s_i s_j / 4 + (Jxy/2) [s_i != s_j] psi(s^ij)/psi(s)]``,
  the definition ``E_x = sum_x' H_xx' Psi_x'/Psi_x`` of Section 3.
* ISGO (Eq. 3): self-normalised weights ``p_x ~ n_x |psi_x|^2/|psi0_x|^2``, local
  energies under the new psi, and the gradient
  ``2 Re[<O* E> - <O*><E>]`` with ``O = d log psi / d theta`` (Eq. 2's garbled
  constant is replaced by this exact derivative of E_v).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp


# ----------------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------------

def num_params(F: int, L: int, tied: bool = True) -> int:
    nW = 1 if tied else L
    return 2 * F + F + nW * (2 * F * F + F) + 2 * (F + 3)


def unpack_theta(theta, F: int, L: int, tied: bool = True) -> dict:
    """Split the flat FP64 vector into named views (layout documented in the C header)."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (num_params(F, L, tied),):
        raise ValueError(f"theta has shape {theta.shape}, expected ({num_params(F, L, tied)},)")
    nW = 1 if tied else L
    out, o = {}, 0

    def take(name, shape):
        nonlocal o
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size

    take("W_e", (2, F))
    take("b_e", (F,))
    take("W", (nW, 2 * F, F))
    take("b", (nW, F))
    take("v_a", (F + 2,))
    take("c_a", ())
    take("v_p", (F + 2,))
    take("c_p", ())
    return out


# ----------------------------------------------------------------------------------
# Graph: the normalised adjacency of Eq. (1)
# ----------------------------------------------------------------------------------

def _check_graph(n: int, edges) -> np.ndarray:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("edge endpoint out of range")
    if np.any(e[:, 0] == e[:, 1]):
        raise ValueError("self-loop")
    key = np.sort(e, axis=1)
    if len(np.unique(key, axis=0)) != len(key):
        raise ValueError("duplicate edge")
    return e


def degrees(n: int, edges) -> np.ndarray:
    e = _check_graph(n, edges)
    return np.bincount(e.ravel(), minlength=n).astype(np.float64)


def normalized_adjacency(n: int, edges, kind: str = "dense"):
    """``D^-1/2 A D^-1/2`` of Eq. (1); A symmetric 0/1 without self-loops."""
    e = _check_graph(n, edges)
    A = np.zeros((n, n))
    A[e[:, 0], e[:, 1]] = 1.0
    A[e[:, 1], e[:, 0]] = 1.0
    d = A.sum(axis=1)
    dinv = np.zeros(n)
    dinv[d > 0] = d[d > 0] ** -0.5
    Ahat = dinv[:, None] * A * dinv[None, :]
    if kind == "dense":
        return Ahat
    if kind == "sparse":
        return sp.csr_matrix(Ahat)
    raise ValueError(kind)


# ----------------------------------------------------------------------------------
# Forward pass (Eq. 1 and the readout of Section 2)
# ----------------------------------------------------------------------------------

def _aggregate(H, n, edges, formulation, cache):
    """Message ``M = A_hat H`` for a batch ``H[B, N, F]``."""
    if formulation == "dense":
        Ahat = cache.setdefault("dense", normalized_adjacency(n, edges, "dense"))
        return np.einsum("ij,bjf->bif", Ahat, H)
    if formulation == "sparse":
        Ahat = cache.setdefault("sparse", normalized_adjacency(n, edges, "sparse"))
        B, N, F = H.shape
        Ht = H.transpose(1, 0, 2).reshape(N, B * F)
        return np.asarray(Ahat @ Ht).reshape(N, B, F).transpose(1, 0, 2)
    if formulation == "edges":
        d = degrees(n, edges)
        M = np.zeros_like(H)
        for i, j in np.asarray(edges, dtype=np.int64):
            w = 1.0 / math.sqrt(d[i] * d[j])
            M[:, i, :] += w * H[:, j, :]
            M[:, j, :] += w * H[:, i, :]
        return M
    raise ValueError(formulation)


LN_EPS = 1e-5   # layer-normalisation epsilon (unstated in the paper; no affine parameters)


def activate(P, act: str = "tanh"):
    """The nonlinearity f of Eq. 1 on the last axis of ``P``.

    ``tanh``; or ``relu_ln``, the paper's own choice (Section 2): ReLU, then a layer
    normalisation over the F features of each node, ``(y - mean y) / sqrt(var y + eps)``
    with the biased variance.  Returns ``(H, aux)``; ``aux = (y, r)`` for ``relu_ln``
    (post-ReLU values and ``r = 1/sqrt(var + eps)``), ``None`` for tanh.
    """
    if act == "tanh":
        return np.tanh(P), None
    if act != "relu_ln":
        raise ValueError(act)
    y = np.maximum(P, 0.0)
    mu = y.mean(axis=-1, keepdims=True)
    var = ((y - mu) ** 2).mean(axis=-1, keepdims=True)
    r = 1.0 / np.sqrt(var + LN_EPS)
    return (y - mu) * r, (y, r)


def activate_vjp(dH, H, aux, act: str = "tanh"):
    """Cotangent of the pre-activation from that of ``H = f(P)`` (same shapes)."""
    if act == "tanh":
        return dH * (1.0 - H ** 2)
    y, r = aux
    # d xhat_i / d y_j = r (delta_ij - 1/F - xhat_i xhat_j / F)
    dy = r * (dH - dH.mean(axis=-1, keepdims=True) - H * (dH * H).mean(axis=-1, keepdims=True))
    return dy * (y > 0.0)


def forward(theta, spins, n: int, edges, F: int, L: int, tied: bool = True,
            formulation: str = "sparse", keep: bool = False, act: str = "tanh"):
    """Evaluate the ansatz on ``spins[B, N]`` in {-1, +1}.

    Returns ``logpsi[B, 2]`` = (log|psi|, phase); with ``keep=True`` also a dict of
    per-layer inputs/outputs for the reverse pass.  ``act`` selects f (``activate``).
    """
    p = unpack_theta(theta, F, L, tied)
    s = np.asarray(spins)
    if s.ndim != 2 or s.shape[1] != n:
        raise ValueError("spins must be [B, N]")
    x = (s.astype(np.int64) + 1) // 2                     # occupation in {0, 1}
    onehot = np.stack([x == 0, x == 1], axis=-1).astype(np.float64)   # [B, N, 2]
    H, aux = activate(onehot @ p["W_e"] + p["b_e"], act)   # embedding
    cache: dict = {}
    Hs, Ms, auxs = [H], [], [aux]
    for l in range(L):
        W = p["W"][0 if tied else l]
        b = p["b"][0 if tied else l]
        M = _aggregate(H, n, edges, formulation, cache)
        P = np.concatenate([M, H], axis=-1) @ W + b        # Eq. (1), message first
        H, aux = activate(P, act)
        Ms.append(M)
        Hs.append(H)
        auxs.append(aux)
    z = np.concatenate([H.sum(axis=1), onehot.sum(axis=1)], axis=-1)   # [B, F+2]
    logabs = z @ p["v_a"] + p["c_a"]
    phase = z @ p["v_p"] + p["c_p"]
    out = np.stack([logabs, phase], axis=-1)
    if keep:
        return out, {"onehot": onehot, "H": Hs, "M": Ms, "z": z, "aux": auxs}
    return out


def logpsi(theta, spins, n, edges, F, L, tied=True, formulation="sparse", chunk=4096, act="tanh"):
    """``forward`` over a large batch in chunks (same arithmetic per row)."""
    s = np.asarray(spins)
    out = np.empty((s.shape[0], 2))
    for a in range(0, s.shape[0], chunk):
        out[a:a + chunk] = forward(theta, s[a:a + chunk], n, edges, F, L, tied, formulation, act=act)
    return out


# ----------------------------------------------------------------------------------
# Local energy (Section 3's E_x for the Heisenberg model)
# ----------------------------------------------------------------------------------

def n_evals(spins, edges) -> int:
    """Number of log-psi evaluations E_loc needs: one per sample plus one per
    anti-aligned bond."""
    s = np.asarray(spins)
    e = np.asarray(edges, dtype=np.int64)
    return int(s.shape[0] + np.sum(s[:, e[:, 0]] != s[:, e[:, 1]]))


def local_energy_generic(logpsi_fn, spins, edges, jz: float = 1.0, jxy: float = 1.0,
                         base=None, batch_target: int = 8192, hb: float = 0.0, cb: float = 0.0):
    """``E(s) = sum_<ij> [jz s_i s_j/4 + hb (s_i + s_j)/4 + cb
                         + (jxy/2)[s_i != s_j] exp(logpsi(s^ij) - logpsi(s))]``.

    The Heisenberg model of Section 3 is ``hb = cb = 0``; the hard-core bosons of
    Eq. 4 map onto this bond form (``oracle.hcb.spin_couplings``).
    ``logpsi_fn(spins[b, N]) -> [b, 2]`` is any ansatz; terms are added in edge-list
    order.  Returns complex ``[B]``.
    """
    s = np.asarray(spins)
    e = np.asarray(edges, dtype=np.int64)
    B = s.shape[0]
    if base is None:
        base = logpsi_fn(s) if B else np.zeros((0, 2))
    base = np.asarray(base, dtype=np.float64)
    out = np.zeros(B, dtype=np.complex128)
    per = max(1, batch_target // max(1, len(e)))
    for a in range(0, B, per):
        rows, cols, confs = [], [], []
        for b in range(a, min(B, a + per)):
            anti = np.nonzero(s[b, e[:, 0]] != s[b, e[:, 1]])[0]
            if anti.size == 0:
                continue
            c = np.repeat(s[b][None, :], anti.size, axis=0)
            ii, jj = e[anti, 0], e[anti, 1]
            r = np.arange(anti.size)
            c[r, ii], c[r, jj] = s[b, jj], s[b, ii]
            rows.append(np.full(anti.size, b))
            cols.append(anti)
            confs.append(c)
        lp = logpsi_fn(np.concatenate(confs)) if confs else np.zeros((0, 2))
        rows = np.concatenate(rows) if rows else np.zeros(0, int)
        o = 0
        for b in range(a, min(B, a + per)):
            si, sj = s[b, e[:, 0]].astype(np.int64), s[b, e[:, 1]].astype(np.int64)
            diag = 0.25 * jz * float(np.sum(si * sj)) + 0.25 * hb * float(np.sum(si + sj)) + cb * len(e)
            k = int(np.sum(rows == b))
            d = lp[o:o + k] - base[b]
            ratio = np.exp(d[:, 0] + 1j * d[:, 1])          # psi(s^ij) / psi(s)
            off = 0.0 + 0.0j
            for t in ratio:                                  # edge-list order
                off += t
            out[b] = diag + 0.5 * jxy * off
            o += k
    return out


def local_energy(theta, spins, n, edges, F, L, tied=True, jz=1.0, jxy=1.0,
                 formulation="sparse", hb=0.0, cb=0.0, act="tanh"):
    """E_loc of the GCN ansatz (complex ``[B]``)."""
    fn = lambda c: logpsi(theta, c, n, edges, F, L, tied, formulation, act=act)
    return local_energy_generic(fn, spins, edges, jz, jxy, hb=hb, cb=cb)


# ----------------------------------------------------------------------------------
# ISGO statistics (Eq. 3) and the reverse pass
# ----------------------------------------------------------------------------------

def isgo_stats(logpsi_old, logpsi_new, eloc, counts=None):
    """Importance weights and centred cotangents for Eq. (3).

    ``r_x = n_x exp(2 Re(lpnew - lpold) - m)`` with the max shift ``m`` (it cancels in
    ``p_x = r_x / sum r``).  Returns ``(stats, cot)`` where ``stats`` holds
    Re E, Im E, variance, ESS, sum r, m, and ``cot[B, 2]`` are the cotangents of
    (log|psi|, phase): ``2 p_x Re(E_x - E)`` and ``2 p_x Im(E_x - E)``.
    """
    old = np.asarray(logpsi_old, dtype=np.float64)
    new = np.asarray(logpsi_new, dtype=np.float64)
    E = np.asarray(eloc, dtype=np.complex128)
    B = E.shape[0]
    n = np.ones(B) if counts is None else np.asarray(counts, dtype=np.float64)
    dlog = 2.0 * (new[:, 0] - old[:, 0])
    finite = bool(np.all(np.isfinite(dlog)) and np.all(np.isfinite(E)) and np.all(np.isfinite(n)))
    m = float(np.max(dlog)) if B else 0.0
    r = n * np.exp(dlog - m)
    S = math.fsum(r)
    p = r / S
    Ebar = complex(math.fsum(p * E.real), math.fsum(p * E.imag))
    dev = E - Ebar
    var = math.fsum(p * np.abs(dev) ** 2)
    ess = S * S / math.fsum(r * r)
    cot = np.stack([2.0 * p * dev.real, 2.0 * p * dev.imag], axis=-1)
    stats = {"e_re": Ebar.real, "e_im": Ebar.imag, "var": var, "ess": ess,
             "sum_r": S, "shift": m, "finite": finite}
    return stats, cot


def logpsi_vjp(theta, spins, cot, n, edges, F, L, tied=True, formulation="sparse", act_fn="tanh"):
    """``g = sum_x cot[x,0] d log|psi(s_x)|/dtheta + cot[x,1] d phase(s_x)/dtheta``.

    Hand-derived reverse pass of ``forward`` (layout of ``g`` = layout of theta).
    """
    p = unpack_theta(theta, F, L, tied)
    cot = np.asarray(cot, dtype=np.float64)
    _, act = forward(theta, spins, n, edges, F, L, tied, formulation, keep=True, act=act_fn)
    g = {k: np.zeros_like(v, dtype=np.float64) for k, v in p.items()}
    ca, cp = cot[:, 0], cot[:, 1]
    z = act["z"]
    g["v_a"] = ca @ z
    g["c_a"] = np.array(ca.sum())
    g["v_p"] = cp @ z
    g["c_p"] = np.array(cp.sum())
    dz = ca[:, None] * p["v_a"][None, :] + cp[:, None] * p["v_p"][None, :]   # [B, F+2]
    Nn = act["H"][0].shape[1]
    dH = np.repeat(dz[:, None, :F], Nn, axis=1)            # d z / d H^L_i = identity
    Ahat = normalized_adjacency(n, edges, "sparse")
    for l in reversed(range(L)):
        wi = 0 if tied else l
        Hin, Hout, M = act["H"][l], act["H"][l + 1], act["M"][l]
        dP = activate_vjp(dH, Hout, act["aux"][l + 1], act_fn)
        X = np.concatenate([M, Hin], axis=-1)              # [B, N, 2F]
        g["W"][wi] += np.einsum("bnk,bnf->kf", X, dP)
        g["b"][wi] += dP.sum(axis=(0, 1))
        dX = dP @ p["W"][wi].T                             # [B, N, 2F]
        dM, dself = dX[..., :F], dX[..., F:]
        B_, N_, _ = dM.shape
        # A_hat is symmetric, so the transpose product is A_hat @ dM again
        dMsum = np.asarray(Ahat @ dM.transpose(1, 0, 2).reshape(N_, B_ * F)).reshape(N_, B_, F).transpose(1, 0, 2)
        dH = dself + dMsum
    dP0 = activate_vjp(dH, act["H"][0], act["aux"][0], act_fn)
    g["W_e"] += np.einsum("bnc,bnf->cf", act["onehot"], dP0)
    g["b_e"] += dP0.sum(axis=(0, 1))
    return np.concatenate([np.atleast_1d(g[k]).ravel() for k in
                           ("W_e", "b_e", "W", "b", "v_a", "c_a", "v_p", "c_p")])


def isgo_grad(theta, spins, logpsi_old, n, edges, F, L, tied=True, counts=None,
              jz=1.0, jxy=1.0, formulation="sparse", hb=0.0, cb=0.0, act="tanh"):
    """One ISGO update's gradient (Eq. 3): new log psi, E_loc under the new psi,
    weights, then the reverse pass with the centred cotangents.

    Returns ``(grad, stats, eloc)``; ``stats`` also carries ``n_evals``.
    """
    new = logpsi(theta, spins, n, edges, F, L, tied, formulation, act=act)
    fn = lambda c: logpsi(theta, c, n, edges, F, L, tied, formulation, act=act)
    E = local_energy_generic(fn, spins, edges, jz, jxy, base=new, hb=hb, cb=cb)
    stats, cot = isgo_stats(logpsi_old, new, E, counts)
    stats["n_evals"] = n_evals(spins, edges)
    g = logpsi_vjp(theta, spins, cot, n, edges, F, L, tied, formulation, act_fn=act)
    return g, stats, E


def sgd_update(theta, grad, alpha):
    """Section 3's update ``w <- w - alpha dE/dw``."""
    return np.asarray(theta, dtype=np.float64) - alpha * np.asarray(grad, dtype=np.float64)
