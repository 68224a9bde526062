"""Pins of the mask-network oracle against brute force and closed forms (CPU).

The oracle's layers are torch library calls; each is checked here against an
independent loop or a closed form, so that a wrong padding, pooling window,
interpolation convention or concatenation order would fail."""
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import mask_oracle as M

DT = torch.float64


def _rng(seed=0):
    return np.random.Generator(np.random.PCG64(seed))


def test_network_size_and_channel_pattern():
    convs = M.conv_list(4, 8)
    assert [c.c_out for c in convs] == [8, 8, 16, 16, 32, 32, 64, 64, 32, 32, 16, 16, 8, 8]
    # skip concatenation widths: upsampled + skip (Table II's 384 = 256 + 128 pattern)
    assert [c.c_in for c in convs if c.name.endswith("a") and c.name.startswith("dec")] == [96, 48, 24]
    weights = sum(c.c_out * c.c_in * 9 for c in convs) + 8 * 9
    assert weights == 121_680
    assert M.param_count(4, 8) == weights + 2 * sum(c.c_out for c in convs) + 1


def test_conv2d_matches_direct_sum():
    r = _rng(1)
    x = torch.tensor(r.normal(size=(2, 3, 5, 6)), dtype=DT)
    w = torch.tensor(r.normal(size=(4, 3, 3, 3)), dtype=DT)
    got = F.conv2d(x, w, padding=1)
    ref = torch.zeros(2, 4, 5, 6, dtype=DT)
    for i in range(2):
        for o in range(4):
            for y in range(5):
                for xx in range(6):
                    s = 0.0
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xi = y + ky - 1, xx + kx - 1
                                if 0 <= yy < 5 and 0 <= xi < 6:
                                    s += float(x[i, c, yy, xi]) * float(w[o, c, ky, kx])
                    ref[i, o, y, xx] = s
    assert torch.allclose(got, ref, atol=1e-12)


def test_batch_norm_uses_batch_statistics():
    r = _rng(2)
    z = torch.tensor(r.normal(3.0, 2.0, size=(4, 3, 5, 5)), dtype=DT)
    gam = torch.tensor([1.0, 2.0, 0.5], dtype=DT)
    bet = torch.tensor([0.0, -1.0, 3.0], dtype=DT)
    _, a = M.conv_bn_relu(z, torch.eye(3, dtype=DT)[:, :, None, None].repeat(1, 1, 3, 3) *
                          torch.tensor([0, 0, 0, 0, 1, 0, 0, 0, 0], dtype=DT).reshape(1, 1, 3, 3),
                          gam, bet, 1e-5)
    for c in range(3):
        v = z[:, c].flatten()
        mu = v.sum() / v.numel()
        var = ((v - mu) ** 2).sum() / v.numel()
        ref = torch.clamp((z[:, c] - mu) / math.sqrt(var + 1e-5) * gam[c] + bet[c], min=0)
        assert torch.allclose(a[:, c], ref, atol=1e-12)


def test_max_pool_matches_windows():
    r = _rng(3)
    x = torch.tensor(r.normal(size=(1, 2, 6, 8)), dtype=DT)
    got = F.max_pool2d(x, 2)
    for c in range(2):
        for y in range(3):
            for xx in range(4):
                assert got[0, c, y, xx] == x[0, c, 2 * y:2 * y + 2, 2 * xx:2 * xx + 2].max()


def _up_weights_1d(n_in):
    """Half-pixel-centre bilinear x2 as an explicit matrix: output o samples
    source position max(0, (o + 0.5) / 2 - 0.5), the upper neighbour clamped."""
    W = np.zeros((2 * n_in, n_in))
    for o in range(2 * n_in):
        s = max(0.0, (o + 0.5) / 2 - 0.5)
        i0 = int(math.floor(s))
        lam = s - i0
        i1 = min(i0 + 1, n_in - 1)
        W[o, i0] += 1 - lam
        W[o, i1] += lam
    return W


def test_upsample_is_separable_half_pixel_bilinear():
    r = _rng(4)
    x = torch.tensor(r.normal(size=(1, 1, 4, 5)), dtype=DT)
    Wy, Wx = _up_weights_1d(4), _up_weights_1d(5)
    ref = Wy @ x[0, 0].numpy() @ Wx.T
    assert np.allclose(M.up2(x)[0, 0].numpy(), ref, atol=1e-12)
    # closed forms: constants stay constant; a ramp i -> i maps to o/2 - 1/4 inside
    ramp = torch.arange(6, dtype=DT).repeat(6, 1)[None, None]
    u = M.up2(ramp)[0, 0, 3]
    assert torch.allclose(u[1:-1], torch.arange(1, 11, dtype=DT) / 2 - 0.25)
    assert float(u[0]) == 0.0 and float(u[-1]) == 5.0
    assert torch.allclose(M.up2(torch.full((1, 1, 3, 3), 2.5, dtype=DT)), torch.tensor(2.5, dtype=DT))


def test_unpack_layout_and_concat_order():
    th = torch.arange(M.param_count(2, 2), dtype=DT)
    P = M.unpack(th, 2, 2)
    w, g, b = P["enc0a"]
    assert w.shape == (2, 1, 3, 3) and float(w[0, 0, 0, 0]) == 0 and float(g[0]) == 18
    assert P["dec0a"][0].shape == (2, 6, 3, 3)
    wh, bh = P["head"]
    assert float(bh[0]) == th.numel() - 1
    # concatenation puts the upsampled deep features first
    x = torch.zeros(1, 8, 8, dtype=DT)
    _, acts = M.forward(x + 1.0, torch.tensor(M.init_params(2, 2), dtype=DT), 2, 2, keep=True)
    assert torch.allclose(acts["cat0"][:, :4], M.up2(acts["enc1b"]))
    assert torch.allclose(acts["cat0"][:, 4:], acts["enc0b"])


def test_mask_is_a_probability_map():
    r = _rng(5)
    x = torch.tensor(r.random((3, 16, 16)), dtype=DT)
    m = M.forward(x, torch.tensor(M.init_params(3, 4, seed=1), dtype=DT), 3, 4)
    assert m.shape == (3, 16, 16) and bool(((m > 0) & (m < 1)).all())


def test_gradient_matches_central_differences():
    r = _rng(6)
    L, base = 2, 2
    x = torch.tensor(r.random((2, 8, 8)), dtype=DT)
    th = torch.tensor(M.init_params(L, base, seed=2), dtype=DT)
    dm = torch.tensor(r.normal(size=(2, 8, 8)), dtype=DT)
    g = M.grad(x, dm, th, L, base)
    v = torch.tensor(r.normal(size=th.numel()), dtype=DT)
    h = 1e-5
    fp = (M.forward(x, th + h * v, L, base) * dm).sum()
    fm = (M.forward(x, th - h * v, L, base) * dm).sum()
    fd = (fp - fm) / (2 * h)
    assert abs(float(fd) - float(g @ v)) <= 1e-6 * max(1.0, abs(float(fd)))


def test_pose_losses_and_adam_closed_forms():
    p = torch.tensor([[0.1, 1.0, -2.0], [0.0, 0.5, 0.5]], dtype=DT)
    t = torch.tensor([[0.0, 0.0, 0.0], [0.2, 0.5, 1.5]], dtype=DT)
    assert abs(float(M.pose_loss(p, t, "l1")) - (3.1 + 1.2) / 2) < 1e-12
    assert abs(float(M.pose_loss(p, t, "l2")) - (0.01 + 1 + 4 + 0.04 + 1) / 2) < 1e-12
    th = torch.tensor([1.0, -2.0, 0.0], dtype=DT)
    g = torch.tensor([0.5, -3.0, 0.0], dtype=DT)
    z = torch.zeros(3, dtype=DT)
    th1, m, v = M.adam_step(th, g, z, z, 1, lr=0.1)
    # the first bias-corrected step moves every weight by lr * g / (|g| + eps)
    assert torch.allclose(th1, th - 0.1 * g / (g.abs() + 1e-8), atol=1e-12)
    assert torch.allclose(m, 0.1 * g) and torch.allclose(v, 0.001 * g * g)


@pytest.mark.parametrize("levels,base", [(1, 8), (4, 8)])
def test_init_is_deterministic(levels, base):
    a, b = M.init_params(levels, base, seed=3), M.init_params(levels, base, seed=3)
    assert a.dtype == np.float32 and a.size == M.param_count(levels, base) and np.array_equal(a, b)
