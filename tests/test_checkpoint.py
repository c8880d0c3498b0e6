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


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_probe_maps_round_trip(tmp_path, dtype):
    g = torch.Generator().manual_seed(3)
    tex = torch.rand(5, 8, 8, 4, generator=g).to(dtype)
    depth = torch.rand(5, 8, 8, generator=g)
    pos = torch.randn(5, 3, generator=g)
    path = str(tmp_path / "maps.safetensors")
    sop.save_probe_maps(path, tex, depth, pos, scene="object", res=8)
    back, meta = sop.load_probe_maps(path)
    assert meta == {"scene": "object", "res": "8"}
    assert back["texels"].dtype == dtype and torch.equal(back["texels"], tex)
    assert torch.equal(back["depth"], depth) and torch.equal(back["probe_pos"], pos)
    sop.save_probe_maps(path, tex)
    back, _ = sop.load_probe_maps(path)
    assert set(back) == {"texels"}


def test_probe_maps_refuse_bad_shapes(tmp_path):
    from safetensors.torch import save_file
    with pytest.raises(ValueError):
        sop.save_probe_maps(str(tmp_path / "a.safetensors"), torch.zeros(2, 4, 4, 3))
    with pytest.raises(ValueError):
        sop.save_probe_maps(str(tmp_path / "b.safetensors"), torch.zeros(2, 4, 4, 4),
                            depth=torch.zeros(2, 4, 5))
    path = str(tmp_path / "c.safetensors")
    save_file({"texels": torch.zeros(2, 4, 4, 4), "depth": torch.zeros(3, 4, 4)}, path)
    with pytest.raises(ValueError):
        sop.load_probe_maps(path)
    save_file({"texels": torch.zeros(2, 4, 4, 4, dtype=torch.float64)}, path)
    with pytest.raises(ValueError):
        sop.load_probe_maps(path)
