"""Model files on the host: a saved model loads back bit for bit with its settings, and a
file of another kind or shape is refused."""
import numpy as np
import pytest


def test_model_file_round_trip(tmp_path):
    import torch

    from paper_2510_05814_amd import checkpoint as ck
    rng = np.random.default_rng(3)
    raw = torch.from_numpy(rng.normal(size=(37, 15)).astype(np.float32))
    raw[4, 5] = float(np.float32(-1e-30))
    p = str(tmp_path / "m.safetensors")
    ck.save_model(p, raw, 3, 1, 200, 120, radius=2.5, box="tight", trunc="render")
    got, info = ck.load_model(p)
    assert torch.equal(got, raw)
    assert info == {"C": 3, "order": 1, "width": 200, "height": 120, "radius": 2.5,
                    "box": "tight", "mode": "smoe", "trunc": "render"}


def test_model_file_checks(tmp_path):
    import torch
    from safetensors.torch import save_file

    from paper_2510_05814_amd import checkpoint as ck
    with pytest.raises(ValueError):
        ck.save_model(str(tmp_path / "a.safetensors"), torch.zeros(4, 9), 3, 1, 8, 8)
    p = str(tmp_path / "b.safetensors")
    save_file({"raw": torch.zeros(4, 15)}, p, metadata={"format": "something-else"})
    with pytest.raises(ValueError):
        ck.load_model(p)
