"""Proposal checkpoints on the host: a save/load round trip keeps parameters, Adam moments,
step count and feature box bit for bit, and a malformed file is refused."""
import pytest
import torch

from paper_2510_07729_amd import _lib as L
from paper_2510_07729_amd import sop


def test_checkpoint_round_trip(tmp_path):
    g = torch.Generator().manual_seed(0)
    mlp = sop.Mlp(torch.randn(L.SOP_MLP_PARAMS, generator=g), [-1.0, -2.0, -0.5],
                  [1.0, 2.0, 0.5])
    mlp.m = torch.randn(L.SOP_MLP_PARAMS, generator=g)
    mlp.v = torch.rand(L.SOP_MLP_PARAMS, generator=g)
    mlp.step = 1234
    path = str(tmp_path / "ck.safetensors")
    mlp.save(path, iteration=77)
    back, meta = sop.Mlp.load(path)
    assert meta["iteration"] == "77" and back.step == 1234
    assert back.lo == mlp.lo and back.hi == mlp.hi
    for a, b in ((back.params, mlp.params), (back.m, mlp.m), (back.v, mlp.v)):
        assert a.dtype == torch.float32 and torch.equal(a, b)


def test_checkpoint_rejects_wrong_shapes(tmp_path):
    from safetensors.torch import save_file
    path = str(tmp_path / "bad.safetensors")
    save_file({"params": torch.zeros(10), "adam_m": torch.zeros(10),
               "adam_v": torch.zeros(10)}, path,
              metadata={"step": "0", "bounds_lo": "[0, 0, 0]", "bounds_hi": "[1, 1, 1]"})
    with pytest.raises(ValueError):
        sop.Mlp.load(path)
