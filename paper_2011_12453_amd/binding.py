"""ctypes binding of ``libgna.so``: argument marshalling only.

Every numeric step runs in the library's HIP kernels.  torch provides device
memory and the stream; inputs are validated for dtype, device, shape and
contiguity here, then passed as raw device pointers.  If the library is absent
the import of this module still works, but creating a ``GNA`` context raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
FP64, FP32, BF16, BF16_1X = 0, 1, 2, 3
PRECISIONS = {"fp64": FP64, "fp32": FP32, "bf16": BF16, "bf16_1x": BF16_1X}
STAT_FIELDS = ("e_re", "e_im", "var", "ess", "sum_r", "shift", "n_evals", "nonfinite")
_STATUS = {0: "OK", 1: "INVALID_ARG", 2: "BAD_GRAPH", 3: "UNSUPPORTED", 4: "OUT_OF_MEMORY",
           5: "HIP_ERROR"}


class GnaError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gna {_STATUS.get(status, status)}: {msg}")
        self.status = status


class _Config(ctypes.Structure):
    _fields_ = [
        ("n_sites", ctypes.c_int32), ("n_edges", ctypes.c_int32),
        ("edges", ctypes.POINTER(ctypes.c_int32)),
        ("n_features", ctypes.c_int32), ("n_layers", ctypes.c_int32), ("tied", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("jz", ctypes.c_double), ("jxy", ctypes.c_double),
        ("max_batch", ctypes.c_int32), ("eloc_mode", ctypes.c_int32),
        ("activation", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("act_budget_bytes", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


_EXPORTS = {
    "gna_init": (ctypes.c_int32, [ctypes.POINTER(_Config), ctypes.POINTER(ctypes.c_void_p)]),
    "gna_destroy": (None, [ctypes.c_void_p]),
    "gna_num_params": (ctypes.c_int64, [ctypes.c_void_p]),
    "gna_last_error": (ctypes.c_char_p, [ctypes.c_void_p]),
    "gna_set_stream": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p]),
    "gna_logpsi": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_void_p]),
    "gna_local_energy": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_void_p]),
    "gna_local_energy_noalloc": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                                  ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "gna_metropolis_sweep": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                              ctypes.c_uint64, ctypes.c_uint64, ctypes.c_void_p]),
    "gna_logpsi_vjp": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    "gna_isgo_grad": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p]),
    "gna_sgd_update": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double]),
    "gna_step": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_void_p]),
    "gna_autotune": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_int32)]),
    "gna_config_info": (ctypes.c_int32, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32]),
    "gna_set_shape": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                       ctypes.c_int32]),
    "gna_group_duplicates": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                              ctypes.c_void_p, ctypes.c_void_p]),
    "gna_set_couplings": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_double]),
    "gna_profile_enable": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32]),
    "gna_profile_read": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]),
}

_LIB = None


def library_path() -> str:
    return os.environ.get("GNA_LIBRARY", os.path.join(_HERE, "libgna.so"))


def load_library():
    """Load ``libgna.so`` once; raise if it is missing (no fallback exists)."""
    global _LIB
    if _LIB is None:
        path = library_path()
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                               "(there is no CPU fallback)")
        lib = ctypes.CDLL(path)
        for name, (res, args) in _EXPORTS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


def _ptr(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class GNA:
    """One library context: a graph, an ansatz shape, a precision and a stream.

    Methods mirror the C entry points (``gna_logpsi`` -> ``logpsi`` ...).  All
    tensors must live on the context's GPU, be contiguous and have the dtypes
    of the C signatures (theta float64, spins int8, log psi float64 [B, 2]).
    """

    def __init__(self, n_sites: int, edges, n_features: int, n_layers: int, tied: bool = True,
                 precision: str | int = "fp64", jz: float = 1.0, jxy: float = 1.0,
                 max_batch: int = 4096, act_budget_bytes: int = 0, device=None, stream=None,
                 eloc_mode: str | int = "full", activation: str | int = "tanh"):
        self._lib = load_library()
        self._ctx = None
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the GNA library runs only on a gfx950 device")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        self._edges = e
        self.n_sites, self.n_edges = int(n_sites), int(e.shape[0])
        self.n_features, self.n_layers, self.tied = int(n_features), int(n_layers), bool(tied)
        self.precision = prec
        self.max_batch = int(max_batch)
        mode = {"full": 0, "incremental": 1}[eloc_mode] if isinstance(eloc_mode, str) else int(eloc_mode)
        self.eloc_mode = mode
        act = {"tanh": 0, "relu_ln": 1}[activation] if isinstance(activation, str) else int(activation)
        self.activation = act
        with torch.cuda.device(self.device):
            st = torch.cuda.current_stream() if stream is None else stream
            self._stream = st
            cfg = _Config(self.n_sites, self.n_edges, e.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                          self.n_features, self.n_layers, int(self.tied), prec, float(jz), float(jxy),
                          self.max_batch, mode, act, 0, int(act_budget_bytes), ctypes.c_void_p(st.cuda_stream))
            out = ctypes.c_void_p()
            status = self._lib.gna_init(ctypes.byref(cfg), ctypes.byref(out))
        if status != 0:
            raise GnaError(status, self._lib.gna_last_error(None).decode())
        self._ctx = out
        self.num_params = int(self._lib.gna_num_params(self._ctx))

    # -- helpers -----------------------------------------------------------------
    def _check(self, status):
        if status != 0:
            raise GnaError(status, self._lib.gna_last_error(self._ctx).decode())

    def _t(self, t, dtype, shape, name):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t

    def _spins(self, spins):
        if spins.dim() != 2:
            raise ValueError("spins must be [B, N]")
        return self._t(spins, torch.int8, (spins.shape[0], self.n_sites), "spins")

    def _theta(self, theta):
        return self._t(theta, torch.float64, (self.num_params,), "theta")

    def _empty(self, shape, dtype=torch.float64):
        return torch.empty(shape, dtype=dtype, device=self.device)

    # -- entry points --------------------------------------------------------------
    def logpsi(self, theta, spins, out=None):
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        out = self._empty((B, 2)) if out is None else self._t(out, torch.float64, (B, 2), "out")
        self._check(self._lib.gna_logpsi(self._ctx, _ptr(theta), _ptr(spins), B, _ptr(out)))
        return out

    def local_energy(self, theta, spins, out=None, n_evals=None):
        """Returns ``(eloc[B, 2], n_evals[1] int64)`` (both on the device)."""
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        out = self._empty((B, 2)) if out is None else self._t(out, torch.float64, (B, 2), "out")
        nev = self._empty((1,), torch.int64) if n_evals is None else self._t(n_evals, torch.int64, (1,), "n_evals")
        self._check(self._lib.gna_local_energy(self._ctx, _ptr(theta), _ptr(spins), B, _ptr(out), _ptr(nev)))
        return out, nev

    def local_energy_noalloc(self, theta, spins, out, n_evals=None):
        """``gna_local_energy_noalloc``: as ``local_energy`` with the library's static
        scratch; ``out`` [B, 2] (and ``n_evals`` [1] int64, optional) are caller-owned."""
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        out = self._t(out, torch.float64, (B, 2), "out")
        if n_evals is not None:
            n_evals = self._t(n_evals, torch.int64, (1,), "n_evals")
        self._check(self._lib.gna_local_energy_noalloc(self._ctx, _ptr(theta), _ptr(spins), B, _ptr(out),
                                                       _ptr(n_evals)))
        return out, n_evals

    def metropolis_sweep(self, theta, spins, logpsi, n_sweeps: int, seed: int, counter_base: int = 0,
                         n_accept=None):
        """Advance the chains in place; returns ``n_accept[B]`` int32."""
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        logpsi = self._t(logpsi, torch.float64, (B, 2), "logpsi")
        acc = self._empty((B,), torch.int32) if n_accept is None else self._t(n_accept, torch.int32, (B,), "n_accept")
        self._check(self._lib.gna_metropolis_sweep(self._ctx, _ptr(theta), _ptr(spins), _ptr(logpsi), B,
                                                   int(n_sweeps), ctypes.c_uint64(seed),
                                                   ctypes.c_uint64(counter_base), _ptr(acc)))
        return acc

    def logpsi_vjp(self, theta, spins, cot, out=None):
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        cot = self._t(cot, torch.float64, (B, 2), "cot")
        out = self._empty((self.num_params,)) if out is None else self._theta(out)
        self._check(self._lib.gna_logpsi_vjp(self._ctx, _ptr(theta), _ptr(spins), B, _ptr(cot), _ptr(out)))
        return out

    def group_duplicates(self, spins, uniq=None, counts=None, n_unique=None):
        """Distinct rows in first-occurrence order with their counts
        (``gna_group_duplicates``).  Returns ``(uniq[B, N], counts[B], n_unique[1])``,
        all on the device; rows past ``n_unique`` repeat the first with count 0."""
        spins = self._spins(spins)
        B = spins.shape[0]
        uniq = self._empty((B, self.n_sites), torch.int8) if uniq is None else \
            self._t(uniq, torch.int8, (B, self.n_sites), "uniq")
        counts = self._empty((B,)) if counts is None else self._t(counts, torch.float64, (B,), "counts")
        n_unique = self._empty((1,), torch.int32) if n_unique is None else \
            self._t(n_unique, torch.int32, (1,), "n_unique")
        self._check(self._lib.gna_group_duplicates(self._ctx, _ptr(spins), B, _ptr(uniq), _ptr(counts),
                                                   _ptr(n_unique)))
        return uniq, counts, n_unique

    def isgo_grad(self, theta, spins, logpsi_old, counts=None, grad=None, stats=None, eloc=None):
        """Returns ``(grad[P], stats[8], eloc[B, 2])``; stats fields: STAT_FIELDS."""
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        logpsi_old = self._t(logpsi_old, torch.float64, (B, 2), "logpsi_old")
        if counts is not None:
            counts = self._t(counts, torch.float64, (B,), "counts")
        grad = self._empty((self.num_params,)) if grad is None else self._theta(grad)
        stats = self._empty((8,)) if stats is None else self._t(stats, torch.float64, (8,), "stats")
        eloc = self._empty((B, 2)) if eloc is None else self._t(eloc, torch.float64, (B, 2), "eloc")
        self._check(self._lib.gna_isgo_grad(self._ctx, _ptr(theta), _ptr(spins), _ptr(logpsi_old),
                                            _ptr(counts), B, _ptr(grad), _ptr(stats), _ptr(eloc)))
        return grad, stats, eloc

    def sgd_update(self, theta, grad, alpha: float):
        theta, grad = self._theta(theta), self._theta(grad)
        self._check(self._lib.gna_sgd_update(self._ctx, _ptr(theta), _ptr(grad), float(alpha)))
        return theta

    def step(self, theta, spins, logpsi, n_sweeps: int, seed: int, counter, lr: float,
             grad=None, stats=None, eloc=None, n_accept=None):
        """One device-resident step (``gna_step``): log psi, sweeps, counter advance, ISGO
        gradient, SGD.  ``counter`` is a device uint64 tensor of one element (int64 dtype).
        Returns ``(grad[P], stats[8], eloc[B, 2], n_accept[B])``."""
        theta, spins = self._theta(theta), self._spins(spins)
        B = spins.shape[0]
        logpsi = self._t(logpsi, torch.float64, (B, 2), "logpsi")
        counter = self._t(counter, torch.int64, (1,), "counter")
        grad = self._empty((self.num_params,)) if grad is None else self._theta(grad)
        stats = self._empty((8,)) if stats is None else self._t(stats, torch.float64, (8,), "stats")
        eloc = self._empty((B, 2)) if eloc is None else self._t(eloc, torch.float64, (B, 2), "eloc")
        acc = self._empty((B,), torch.int32) if n_accept is None else self._t(n_accept, torch.int32, (B,), "n_accept")
        self._check(self._lib.gna_step(self._ctx, _ptr(theta), _ptr(spins), _ptr(logpsi), B, int(n_sweeps),
                                       ctypes.c_uint64(seed), _ptr(counter), float(lr), _ptr(grad),
                                       _ptr(stats), _ptr(eloc), _ptr(acc)))
        return grad, stats, eloc, acc

    def autotune(self, theta, spins) -> dict:
        """Measure the incremental kernels' shapes on this batch and keep the fastest
        (``gna_autotune``; synchronises).  Returns the choice."""
        theta, spins = self._theta(theta), self._spins(spins)
        out = (ctypes.c_int32 * 8)()
        self._check(self._lib.gna_autotune(self._ctx, _ptr(theta), _ptr(spins), spins.shape[0], out))
        return {"jobs_in_flight": out[0], "waves": out[1], "samples_per_xcd": out[2], "us_per_call": out[3],
                "sweep_jobs_in_flight": out[4], "sweep_waves": out[5], "sweep_tiles_per_wave": out[6],
                "sweep_us_per_call": out[7]}

    def set_shape(self, jobs_in_flight: int, waves: int, samples_per_xcd: int = 2, which: str = "both"):
        """Pin the incremental kernels' shape (``gna_set_shape``); which: "eloc",
        "sweep" or "both"."""
        w = {"eloc": 1, "sweep": 2, "both": 3}[which]
        self._check(self._lib.gna_set_shape(self._ctx, w, int(jobs_in_flight), int(waves), int(samples_per_xcd)))

    def config_info(self) -> dict:
        """Shape in use (``gna_config_info``)."""
        v = (ctypes.c_int32 * 11)()
        if self._lib.gna_config_info(self._ctx, v, 11) != 11:
            raise GnaError(1, "gna_config_info failed")
        keys = ("eloc_mode", "jobs_in_flight", "waves", "tiles_per_wave", "samples_per_xcd", "precision",
                "features", "layers", "sweep_jobs_in_flight", "sweep_waves", "sweep_tiles_per_wave")
        return dict(zip(keys, list(v)))

    def set_couplings(self, jz: float, jxy: float, hb: float = 0.0, cb: float = 0.0):
        """Bond Hamiltonian ``jz s_i s_j/4 + hb (s_i + s_j)/4 + cb + (jxy/2)[s_i != s_j] swap``."""
        self._check(self._lib.gna_set_couplings(self._ctx, float(jz), float(jxy), float(hb), float(cb)))

    def set_hard_core_bosons(self, t: float, V: float):
        """The hard-core bosons of Eq. 4 (occupation n = (1 + s)/2)."""
        self.set_couplings(V, -2.0 * t, V, V / 4.0)

    def set_stream(self, stream):
        """Enqueue later calls on ``stream`` (a torch.cuda.Stream), e.g. a graph-capture stream."""
        self._check(self._lib.gna_set_stream(self._ctx, ctypes.c_void_p(stream.cuda_stream)))
        self._stream = stream

    def profile_enable(self, on: bool = True):
        """Bracket every launch with HIP events on the context's stream."""
        self._check(self._lib.gna_profile_enable(self._ctx, int(bool(on))))

    def profile_read(self) -> dict:
        """``{kernel: (launches, total_ms)}`` since the last read (waits for the stream)."""
        cap = 32
        names = ctypes.create_string_buffer(64 * cap)
        launches = (ctypes.c_int64 * cap)()
        total = (ctypes.c_double * cap)()
        n = self._lib.gna_profile_read(self._ctx, cap, names, launches, total)
        if n < 0:
            raise GnaError(5, "gna_profile_read failed")
        raw = names.raw
        return {raw[64 * k:64 * k + 64].split(b"\0")[0].decode(): (int(launches[k]), float(total[k]))
                for k in range(min(n, cap))}

    def close(self):
        if self._ctx is not None:
            self._lib.gna_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LogPsi(torch.autograd.Function):
    """``LogPsi.apply(gna, theta, spins) -> [B, 2]`` with the hand-written reverse pass."""

    @staticmethod
    def forward(ctx, gna: GNA, theta, spins):
        ctx.gna = gna
        ctx.save_for_backward(theta, spins)
        return gna.logpsi(theta.detach(), spins)

    @staticmethod
    def backward(ctx, grad_out):
        theta, spins = ctx.saved_tensors
        g = ctx.gna.logpsi_vjp(theta.detach(), spins, grad_out.contiguous().to(torch.float64))
        return None, g, None
