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


def test_blank_mask_fallback_policy():
    """A pair whose network output has all but blanked a scan falls back to
    the unmasked pose; the other pairs keep the masked one."""
    masked = torch.tensor([[0.1, 1.0, 2.0], [0.2, 3.0, 4.0], [0.3, 5.0, 6.0]])
    plain = torch.tensor([[9.1, 9.0, 9.0], [9.2, 9.0, 9.0], [9.3, 9.0, 9.0]])
    m_f = torch.rand(3, 8, 8) * 0.5 + 0.25
    m_g = m_f.clone()
    m_g[1].zero_()                      # forced zero mask on pair 1's second scan
    blank = train.blank_masks(m_f.mean(dim=(1, 2)), m_g.mean(dim=(1, 2)), 1e-3)
    assert blank.tolist() == [False, True, False]
    out = train.fallback_poses(masked, plain, blank)
    assert torch.equal(out[0], masked[0]) and torch.equal(out[2], masked[2])
    assert torch.equal(out[1], plain[1])
