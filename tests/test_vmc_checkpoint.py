"""Checkpoint files of the sampling loop (host logic only): round trip and the
compatibility checks."""
import numpy as np
import pytest
import torch

from paper_2011_12453_amd.vmc import load_checkpoint, save_checkpoint, transfer_theta


class _Ctx:   # the attributes the checkpoint helpers read from a context
    def __init__(self, n, F=16, L=2, tied=True, act=0):
        self.n_sites, self.n_features, self.n_layers, self.tied, self.activation = n, F, L, tied, act
        self.device = torch.device("cpu")


def test_round_trip(tmp_path):
    g = _Ctx(12)
    th = torch.from_numpy(np.random.default_rng(0).normal(size=330))
    sp = torch.from_numpy(np.where(np.random.default_rng(1).random((8, 12)) < 0.5, -1, 1).astype(np.int8))
    p = str(tmp_path / "c.npz")
    save_checkpoint(p, g, th, sp, 2 ** 40 + 3, 7)
    d = load_checkpoint(p, g)
    assert torch.equal(d["theta"], th) and torch.equal(d["spins"], sp)
    assert d["counter"] == 2 ** 40 + 3 and d["iteration"] == 7


@pytest.mark.parametrize("other", [dict(F=32), dict(L=3), dict(tied=False), dict(act=1)])
def test_incompatible_context_rejected(tmp_path, other):
    p = str(tmp_path / "c.npz")
    save_checkpoint(p, _Ctx(12), torch.zeros(4, dtype=torch.float64), torch.ones((2, 12), dtype=torch.int8), 0, 0)
    kw = dict(F=16, L=2, tied=True, act=0)
    kw.update(other)
    with pytest.raises(ValueError):
        load_checkpoint(p, _Ctx(12, **kw))
    with pytest.raises(ValueError):
        load_checkpoint(p, _Ctx(36))
    with pytest.raises(ValueError):
        transfer_theta(torch.zeros(4, dtype=torch.float64), _Ctx(12), _Ctx(432, **kw))


def test_transfer_keeps_values():
    th = torch.arange(10, dtype=torch.float64)
    out = transfer_theta(th, _Ctx(12), _Ctx(432))
    assert torch.equal(out, th) and out.data_ptr() != th.data_ptr()
