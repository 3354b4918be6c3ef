"""Checkpoint / resume of the optimisation loop: the state file round-trips on
the CPU (tensors, Adam moments and step counts, level, step, history), loads
without executing anything from the file, and an optimiser restored from it
continues exactly as the uninterrupted one."""
import os
import tempfile

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2012_03939_amd.optimise import load_checkpoint, save_checkpoint


def _problem(seed=0):
    g = torch.Generator().manual_seed(seed)
    V = torch.randn(10, 3, generator=g).requires_grad_(True)
    M = torch.rand(8, 7, generator=g).requires_grad_(True)
    opt = torch.optim.Adam([{"params": [V], "lr": 1e-2}, {"params": [M], "lr": 1e-1}])
    return V, M, opt


def _step(V, M, opt, i):
    opt.zero_grad(set_to_none=True)
    loss = ((V - 0.1 * i) ** 2).sum() + ((M - 0.5) ** 3).abs().sum()
    loss.backward()
    opt.step()


def test_checkpoint_round_trip_and_resume():
    F = torch.randint(0, 10, (8, 3), dtype=torch.int32)
    V, M, opt = _problem()
    for i in range(3):
        _step(V, M, opt, i)
    path = os.path.join(tempfile.mkdtemp(), "ckpt.pt")
    hist = {"times": [0.1, 0.2, 0.3], "l2": [3.0, 2.0, 1.5], "faces": [8]}
    save_checkpoint(path, 1, 2, V, M, F, opt, hist)
    assert not os.path.exists(path + ".tmp")
    for i in range(3, 6):                       # the uninterrupted run goes on
        _step(V, M, opt, i)
    ck = load_checkpoint(path)
    assert ck["level"] == 1 and ck["step"] == 2
    assert ck["history"] == hist
    assert torch.equal(ck["F"], F)
    V2 = ck["V"].clone().requires_grad_(True)
    M2 = ck["M"].clone().requires_grad_(True)
    opt2 = torch.optim.Adam([{"params": [V2], "lr": 1e-2}, {"params": [M2], "lr": 1e-1}])
    opt2.load_state_dict(ck["opt"])
    assert opt2.state[V2]["step"] == 3
    for i in range(3, 6):
        _step(V2, M2, opt2, i)
    assert torch.equal(V2.detach(), V.detach()) and torch.equal(M2.detach(), M.detach())


def test_checkpoint_rejects_other_files():
    path = os.path.join(tempfile.mkdtemp(), "other.pt")
    torch.save({"V": torch.zeros(3)}, path)
    with pytest.raises(ValueError):
        load_checkpoint(path)
