"""save_state / load_state on the host: tensors keep their values and dtypes,
numbers come back as numbers, and a file holding pickled objects is refused."""
import numpy as np
import pytest
import torch

from paper_0706_3060_amd import nbody as nb


def test_state_round_trip(tmp_path):
    g = torch.Generator().manual_seed(5)
    pos = torch.randn(37, 3, dtype=torch.float64, generator=g)
    steps = torch.arange(7, dtype=torch.int64)
    path = tmp_path / "s.npz"
    nb.save_state(path, pos=pos, steps=steps, t=0.125, step=50, seed=44)
    st = nb.load_state(path, device="cpu")
    assert torch.equal(st["pos"], pos) and st["pos"].dtype == torch.float64
    assert torch.equal(st["steps"], steps) and st["steps"].dtype == torch.int64
    assert st["pos"].is_contiguous()
    assert st["t"] == 0.125 and st["step"] == 50 and st["seed"] == 44
    assert isinstance(st["step"], int) and isinstance(st["t"], float)


def test_state_refuses_objects(tmp_path):
    with pytest.raises(ValueError):
        nb.save_state(tmp_path / "bad.npz", x={"a": 1})
    path = tmp_path / "pickled.npz"
    np.savez(path, x=np.array([{"a": 1}], dtype=object))
    with pytest.raises(ValueError):
        nb.load_state(path, device="cpu")
