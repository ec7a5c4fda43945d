"""The fit's checkpoint file (host side): widths, Adam's moments and step
count, and the history survive a save/load round trip exactly."""
import json

import pytest


def test_state_round_trip(tmp_path):
    torch = pytest.importorskip("torch")
    from paper_2601_01210_amd import autograd as AG
    st = {"step": torch.tensor(7.0),
          "exp_avg": torch.tensor([0.1234567890123, -2.5e-7], dtype=torch.float64),
          "exp_avg_sq": torch.tensor([1e-12, 3.0000000000000004], dtype=torch.float64)}
    hist = [{"step": 6, "loss": 0.1875, "sigma_s": 2.05, "sigma_r": 39.95, "targets": 9}]
    p = str(tmp_path / "s.json")
    AG.save_state(p, 2.0500000000000003, 39.95, hist, st, 7)
    back = AG.load_state(p)
    assert back["sigma_s"] == 2.0500000000000003 and back["sigma_r"] == 39.95
    assert back["step"] == 7 and back["adam"]["step"] == 7
    assert back["adam"]["exp_avg"] == st["exp_avg"].tolist()
    assert back["adam"]["exp_avg_sq"] == st["exp_avg_sq"].tolist()
    assert back["history"] == hist
    assert not (tmp_path / "s.json.tmp").exists()
    json.loads(open(p).read())


def test_state_without_adam_moments(tmp_path):
    from paper_2601_01210_amd import autograd as AG
    p = str(tmp_path / "s.json")
    AG.save_state(p, 1.0, 2.0, [])
    back = AG.load_state(p)
    assert back["step"] == 0 and back["adam"]["step"] == 0
