"""Trainer checkpoints on the CPU: a state written by save_checkpoint comes back
field for field through load_checkpoint (weights_only, no code in the file),
with the caller's extra values such as a generator state, and malformed states
are refused."""
import numpy as np
import pytest
import torch

from paper_2203_00459_amd import train


def _state(n=1000, nbn=32, seed=0):
    g = torch.Generator().manual_seed(seed)
    return {"params": torch.randn(n, generator=g), "adam_m": torch.randn(n, generator=g),
            "adam_v": torch.rand(n, generator=g), "adam_step": 17, "bn_running": torch.rand(2 * nbn, generator=g),
            "use_mask": True, "config": {"levels": 4, "base": 8, "lr": 1e-3, "loss": 1, "seed": 0}}


def test_checkpoint_round_trip(tmp_path):
    st = _state()
    rng = np.random.Generator(np.random.PCG64(5))
    rng.random(3)
    path = str(tmp_path / "ckpt.pt")
    train.save_checkpoint(path, st, extra={"rng": rng.bit_generator.state, "epoch": 3})
    back = train.load_checkpoint(path)
    for k in ("params", "adam_m", "adam_v", "bn_running"):
        assert torch.equal(back[k], st[k]), k
    assert back["adam_step"] == 17 and back["use_mask"] is True and back["config"] == st["config"]
    assert back["extra"]["epoch"] == 3
    r2 = np.random.Generator(np.random.PCG64(0))
    r2.bit_generator.state = back["extra"]["rng"]
    assert np.array_equal(r2.random(4), rng.random(4))       # the data order resumes where it stopped
    train.check_state(back, 1000, 64)


def test_malformed_states_are_refused():
    st = _state()
    with pytest.raises(ValueError):
        train.check_state(st, 999, 64)
    with pytest.raises(ValueError):
        train.check_state(st, 1000, 63)
    bad = dict(st, adam_v=st["adam_v"].double())
    with pytest.raises(ValueError):
        train.check_state(bad, 1000, 64)
    bad = dict(st)
    del bad["adam_step"]
    with pytest.raises(ValueError):
        train.check_state(bad, 1000, 64)
