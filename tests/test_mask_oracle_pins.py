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


def test_input_gradient_matches_central_differences():
    """The input gradient (what fmbym_mask_bwd returns as d_x) against central
    differences of the FP64 forward, one scan pixel at a time (a perturbation of
    every pixel at once can carry a ReLU or max-pool switch inside +-h)."""
    r = _rng(16)
    L, base = 2, 2
    x = torch.tensor(r.random((2, 8, 8)), dtype=DT)
    th = torch.tensor(M.init_params(L, base, seed=3), dtype=DT)
    dm = torch.tensor(r.normal(size=(2, 8, 8)), dtype=DT)
    g = M.grad_input(x, dm, th, L, base)
    assert g.shape == x.shape
    h = 1e-5
    for idx in [(0, 3, 3), (1, 0, 0), (0, 7, 2), (1, 5, 6), (0, 0, 7), (1, 7, 7)]:
        e = torch.zeros_like(x)
        e[idx] = 1.0
        fd = ((M.forward(x + h * e, th, L, base) - M.forward(x - h * e, th, L, base)) * dm).sum() / (2 * h)
        assert abs(float(fd) - float(g[idx])) <= 1e-6 * max(1.0, abs(float(fd))), idx


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


# ------------------------------------------------------------------ bf16 storage

def _bf16_rne_bits(x32: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (8 significant bits), ties to
    the even significand, by integer arithmetic on the IEEE-754 bit patterns:
    add 0x7FFF plus the lowest kept bit, then clear the 16 dropped bits."""
    u = x32.astype(np.float32).view(np.uint32).astype(np.uint64)
    r = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def test_bf16_rounds_to_nearest_even_on_chosen_values():
    # (input, bfloat16 value): the significand keeps 8 bits (7 stored); ties go to
    # the even significand; the stored value is that of the input rounded to FP32
    # first (the GPU rounds its FP32 results), so 1 + 2^-8 + 2^-40 is a tie.
    cases = [
        (1.0 + 2.0 ** -9, 1.0),                          # below the half-way point
        (1.0 + 2.0 ** -8, 1.0),                          # tie, 1.0 is even
        (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),          # tie, rounds up to the even neighbour
        (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),  # just above the tie
        (1.0 + 2.0 ** -8 + 2.0 ** -40, 1.0),             # FP32 rounding makes it a tie
        (-(1.0 + 2.0 ** -8), -1.0),
        (255.5, 256.0),                                  # 255 + 1/2 has 9 significant bits: tie to 256
        (257.0, 256.0),                                  # tie between 256 and 258, 256 is even
        (70000.0, 70144.0),                              # beyond the FP16 range, exact bf16 step 512
        (2.0 ** -130, 2.0 ** -130),                      # subnormal, representable
        (1.5 * 2.0 ** -133, 2.0 ** -132),                # subnormal tie goes to the even count 2
        (2.0 ** -134, 0.0),                              # half the smallest subnormal: tie to zero
        (3.0e38, 3.00405527047391e38),
    ]
    x = torch.tensor([c[0] for c in cases], dtype=DT)
    got = M.bf16(x).tolist()
    for (inp, want), g in zip(cases, got):
        assert g == want, (inp, g, want)
    assert torch.equal(M.bf16(x, on=False), x)


def test_bf16_matches_bit_arithmetic_over_exponents():
    r = _rng(11)
    mant = r.random(200_000) + 1.0
    expo = r.integers(-140, 120, size=mant.size).astype(np.float64)
    sign = np.where(r.random(mant.size) < 0.5, -1.0, 1.0)
    x32 = (sign * mant * np.exp2(expo)).astype(np.float32)
    want = _bf16_rne_bits(x32).astype(np.float64)
    got = M.bf16(torch.tensor(x32.astype(np.float64), dtype=DT)).numpy()
    assert np.array_equal(got, want)


def test_bf16_has_identity_derivative():
    x = torch.tensor([1.0 + 2.0 ** -8, 3.3, -7.1], dtype=DT, requires_grad=True)
    (M.bf16(x) * torch.tensor([1.0, 2.0, 3.0], dtype=DT)).sum().backward()
    assert torch.equal(x.grad, torch.tensor([1.0, 2.0, 3.0], dtype=DT))


# ------------------------------------------ running statistics and inference mode

def _delta_net(levels, base, scale_a, scale_b, gam, bet, head_w, head_b):
    """Flat parameters of a one-level, one-channel net whose convolutions are
    centre taps: enc0a multiplies by scale_a, enc0b by scale_b, the head by head_w."""
    assert (levels, base) == (1, 1)
    def tap(s):
        w = np.zeros(9)
        w[4] = s
        return w
    th = np.concatenate([tap(scale_a), [gam[0]], [bet[0]], tap(scale_b), [gam[1]], [bet[1]],
                         tap(head_w), [head_b]])
    assert th.size == M.param_count(1, 1)
    return torch.tensor(th, dtype=DT)


def test_running_stats_momentum_and_unbiased_variance_by_hand():
    r = _rng(12)
    x = r.normal(0.5, 1.2, size=(2, 3, 3))
    th = _delta_net(1, 1, 1.0, 2.0, (1.5, 0.7), (-0.2, 0.1), 1.0, 0.0)
    rm0 = torch.tensor([0.3, -0.1], dtype=DT)
    rv0 = torch.tensor([2.0, 0.5], dtype=DT)
    rm, rv = M.running_stats(torch.tensor(x, dtype=DT), th, 1, 1, rm0, rv0, momentum=0.1)
    # by hand: z1 = x; a1 = relu(BN(z1)) with the biased batch variance; z2 = 2 a1
    v = x.reshape(-1)
    N = v.size
    mu1 = sum(v) / N
    var1_b = sum((t - mu1) ** 2 for t in v) / N
    var1_u = sum((t - mu1) ** 2 for t in v) / (N - 1)
    a1 = [max(0.0, (t - mu1) / math.sqrt(var1_b + 1e-5) * 1.5 - 0.2) for t in v]
    z2 = [2.0 * t for t in a1]
    mu2 = sum(z2) / N
    var2_u = sum((t - mu2) ** 2 for t in z2) / (N - 1)
    want_m = [0.9 * 0.3 + 0.1 * mu1, 0.9 * -0.1 + 0.1 * mu2]
    want_v = [0.9 * 2.0 + 0.1 * var1_u, 0.9 * 0.5 + 0.1 * var2_u]
    assert np.allclose(rm.numpy(), want_m, rtol=0, atol=1e-13)
    assert np.allclose(rv.numpy(), want_v, rtol=0, atol=1e-13)


def test_forward_eval_is_inference_batchnorm_and_relu_by_hand():
    r = _rng(13)
    x = r.normal(0.0, 1.0, size=(2, 4, 4))
    gam, bet = (1.3, 0.8), (-0.4, 0.25)
    th = _delta_net(1, 1, 0.5, -1.5, gam, bet, 2.0, -0.3)
    rm = torch.tensor([0.2, 0.6], dtype=DT)
    rv = torch.tensor([0.9, 1.7], dtype=DT)
    m = M.forward_eval(torch.tensor(x, dtype=DT), th, 1, 1, rm, rv).numpy()
    eps = 1e-5
    want = np.empty_like(x)
    clipped = 0
    for idx in np.ndindex(*x.shape):
        z1 = 0.5 * x[idx]
        a1 = (z1 - 0.2) / math.sqrt(0.9 + eps) * gam[0] + bet[0]
        clipped += a1 < 0
        a1 = max(0.0, a1)
        z2 = -1.5 * a1
        a2 = (z2 - 0.6) / math.sqrt(1.7 + eps) * gam[1] + bet[1]
        clipped += a2 < 0
        a2 = max(0.0, a2)
        want[idx] = 1.0 / (1.0 + math.exp(-(2.0 * a2 - 0.3)))
    assert clipped > 0          # the case exercises the ReLU
    assert np.allclose(m, want, rtol=0, atol=1e-14)


def test_forward_eval_on_the_batch_statistics_is_the_training_forward():
    # BatchNorm on running statistics equal to the batch's (biased variance, as
    # the training normalisation uses) is the training-mode layer, at every depth
    r = _rng(14)
    L, base = 3, 4
    x = torch.tensor(r.random((3, 16, 16)), dtype=DT)
    th = torch.tensor(M.init_params(L, base, seed=4), dtype=DT)
    m, acts = M.forward(x, th, L, base, keep=True)
    means, vars_ = [], []
    for c in M.conv_list(L, base):
        mu, var = M.batch_stats(acts[f"{c.name}.z"])
        means.append(mu)
        vars_.append(var)
    got = M.forward_eval(x, th, L, base, torch.cat(means), torch.cat(vars_))
    assert torch.allclose(got, m, rtol=0, atol=1e-12)
    # and running statistics that differ from the batch's change the mask
    other = M.forward_eval(x, th, L, base, torch.cat(means) + 0.1, torch.cat(vars_))
    assert float((other - m).abs().max()) > 1e-3


def test_quant_forward_eval_on_the_batch_statistics_is_the_quant_training_forward():
    # the same identity with BF16 storage: on the statistics of the stored z,
    # inference rounds at the training forward's points and gives its masks;
    # and the rounding is there (the quant masks differ from the exact ones)
    r = _rng(16)
    L, base = 3, 4
    x = torch.tensor(r.random((3, 16, 16)) * 3.0, dtype=DT)
    th = torch.tensor(M.init_params(L, base, seed=5), dtype=DT)
    m, acts = M.forward(x, th, L, base, keep=True, quant=True)
    means, vars_ = [], []
    for c in M.conv_list(L, base):
        mu, var = M.batch_stats(acts[f"{c.name}.z"])
        means.append(mu)
        vars_.append(var)
    got = M.forward_eval(x, th, L, base, torch.cat(means), torch.cat(vars_), quant=True)
    assert torch.allclose(got, m, rtol=0, atol=1e-12)
    exact = M.forward_eval(x, th, L, base, torch.cat(means), torch.cat(vars_))
    assert float((exact - m).abs().max()) > 1e-5


def test_quant_forward_rounds_at_the_documented_points_by_hand():
    # one level, centre taps: the stored values are bf16(x), bf16(w), bf16(z) and
    # bf16(relu(BN(z))) with BN on the stored z; the head stays unrounded
    r = _rng(15)
    x = r.random((2, 3, 3)) * 3.0
    gam, bet = (1.1, 0.9), (0.05, -0.02)
    wa, wb = 1.0 + 2.0 ** -6 + 2.0 ** -9, 0.7
    th = _delta_net(1, 1, wa, wb, gam, bet, 1.7, 0.1)
    q = lambda v: float(_bf16_rne_bits(np.array([v], dtype=np.float32))[0])
    N = x.size
    z1 = [q(q(t) * q(wa)) for t in x.reshape(-1)]
    mu = sum(z1) / N
    var = sum((t - mu) ** 2 for t in z1) / N
    a1 = [q(max(0.0, (t - mu) / math.sqrt(var + 1e-5) * gam[0] + bet[0])) for t in z1]
    z2 = [q(t * q(wb)) for t in a1]
    mu = sum(z2) / N
    var = sum((t - mu) ** 2 for t in z2) / N
    a2 = [q(max(0.0, (t - mu) / math.sqrt(var + 1e-5) * gam[1] + bet[1])) for t in z2]
    want = np.array([1.0 / (1.0 + math.exp(-(1.7 * t + 0.1))) for t in a2]).reshape(x.shape)
    got = M.forward(torch.tensor(x, dtype=DT), th, 1, 1, quant=True).numpy()
    assert np.allclose(got, want, rtol=0, atol=1e-12)
    exact = M.forward(torch.tensor(x, dtype=DT), th, 1, 1).numpy()
    assert np.abs(exact - want).max() > 1e-4     # the rounding is visible


# ------------------------------------------------ Table II's dual-input network

TABLE_II = [  # (c_in, c_out) of every convolution, encoder then decoder, then the head
    (2, 8), (8, 8), (8, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128),
    (128, 256), (256, 256),
    (384, 128), (128, 128), (192, 64), (64, 64), (96, 32), (32, 32), (48, 16), (16, 16), (24, 8), (8, 8),
]


def test_dual_network_is_table_ii():
    """6 levels, 8 -> 256 channels, two scans in and two masks out: the channel list
    written out by hand from the table, about 1.97 M convolution weights."""
    convs = M.conv_list(6, 8, 2)
    assert [(c.c_in, c.c_out) for c in convs] == TABLE_II
    n_conv = sum(ci * co * 9 for ci, co in TABLE_II) + 8 * 2 * 9
    assert n_conv == 1_965_024
    bn = sum(2 * co for _, co in TABLE_II)
    assert M.param_count(6, 8, 2) == n_conv + bn + 2
    th = torch.tensor(M.init_params(6, 8, seed=0, ch=2), dtype=DT)
    assert th.numel() == M.param_count(6, 8, 2)
    P = M.unpack(th, 6, 8, 2)
    assert P["head"][0].shape == (2, 8, 3, 3) and P["head"][1].shape == (2,)


def test_dual_network_channel_order_against_the_single_channel_network():
    """A dual net whose first convolution ignores input channel 1 and whose two head
    rows are equal returns two identical masks, each the one-channel network's mask of
    channel 0 with the same weights: input channel 0 is the first scan, head row k is
    mask k, and nothing else mixes the channels."""
    r = _rng(21)
    L, base = 3, 4
    th1 = M.init_params(L, base, seed=5)
    P1 = M.unpack(torch.tensor(th1, dtype=DT), L, base)
    parts = []
    for c in M.conv_list(L, base, 2):
        w, g, b = P1[c.name]
        if c.name == "enc0a":
            w2 = torch.zeros(c.c_out, 2, 3, 3, dtype=DT)
            w2[:, 0] = w[:, 0]
            w = w2
        parts += [w.reshape(-1), g, b]
    wh, bh = P1["head"]
    parts += [torch.cat([wh, wh]).reshape(-1), torch.cat([bh, bh])]
    th2 = torch.cat(parts)
    x = torch.tensor(r.random((3, 16, 16)), dtype=DT)
    y = torch.tensor(r.random((3, 16, 16)), dtype=DT)
    m1 = M.forward(x, torch.tensor(th1, dtype=DT), L, base)
    m2 = M.forward(torch.stack([x, y], dim=1), th2, L, base, ch=2)
    assert m2.shape == (3, 2, 16, 16)
    np.testing.assert_allclose(m2[:, 0].numpy(), m1.numpy(), atol=1e-12)
    np.testing.assert_allclose(m2[:, 1].numpy(), m1.numpy(), atol=1e-12)
    # and a different second scan changes nothing
    m3 = M.forward(torch.stack([x, 2 * y + 1], dim=1), th2, L, base, ch=2)
    np.testing.assert_allclose(m3.numpy(), m2.numpy(), atol=1e-12)
