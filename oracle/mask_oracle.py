"""FP64 CPU oracle of the learned mask network and its training step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library.

What it computes (Section III-E): a U-Net h_alpha maps each scan to a mask in
(0, 1)^(n x n) (Eq. 10), the search runs on the masked scans (Eq. 11-12) and
the network is trained on the pose error (Eq. 13) with Adam.  The layer
pattern follows Table II, sized down to the network the build trains: per
level two 3x3 convolutions (padding 1, no bias), each followed by BatchNorm
(batch statistics, eps 1e-5) and ReLU; 2x2 max-pooling between encoder
levels; bilinear x2 upsampling (half-pixel centres, edge clamped) and
concatenation [upsampled, skip] in the decoder; a 3x3 head convolution with
bias and a sigmoid.  Channels double per level from ``base``.  ``ch`` is the
number of input and output channels: 1 for the network whose two scans of a
pair go through the same weights one at a time, 2 for Table II's dual-input
network, which sees both scans of a pair stacked as channels (f, g) and
returns both masks (m_f, m_g).

Every layer is a plain torch-CPU FP64 library call (conv2d, batch_norm,
max_pool2d, interpolate, sigmoid); gradients come from FP64 autograd.  The
pins in tests/test_mask_oracle_pins.py check those calls against brute-force
loops and closed forms.

Flat parameter vector (the library's documented layout, restated here):
for each convolution in order enc0a, enc0b, enc1a, enc1b, ..., dec(L-2)a,
dec(L-2)b, ..., dec0a, dec0b: weight [c_out][c_in][3][3], then gamma [c_out],
then beta [c_out]; finally the head weight [ch][base][3][3] and its bias [ch].
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch
import torch.nn.functional as F

DT = torch.float64


@dataclasses.dataclass(frozen=True)
class Conv:
    name: str
    c_in: int
    c_out: int
    level: int


def conv_list(levels: int, base: int, in_ch: int = 1) -> list[Conv]:
    """The network's convolutions in parameter order."""
    ch = [base << l for l in range(levels)]
    out = []
    for l in range(levels):
        out.append(Conv(f"enc{l}a", in_ch if l == 0 else ch[l - 1], ch[l], l))
        out.append(Conv(f"enc{l}b", ch[l], ch[l], l))
    for l in range(levels - 2, -1, -1):
        out.append(Conv(f"dec{l}a", ch[l + 1] + ch[l], ch[l], l))
        out.append(Conv(f"dec{l}b", ch[l], ch[l], l))
    return out


def param_count(levels: int, base: int, ch: int = 1) -> int:
    return sum(c.c_out * c.c_in * 9 + 2 * c.c_out for c in conv_list(levels, base, ch)) + ch * (base * 9 + 1)


def unpack(theta: torch.Tensor, levels: int, base: int, ch: int = 1) -> dict:
    """Views of the flat parameter vector: {name: (w, gamma, beta)}, 'head': (w, b)."""
    out, o = {}, 0
    for c in conv_list(levels, base, ch):
        nw = c.c_out * c.c_in * 9
        w = theta[o:o + nw].reshape(c.c_out, c.c_in, 3, 3)
        o += nw
        gam = theta[o:o + c.c_out]
        o += c.c_out
        bet = theta[o:o + c.c_out]
        o += c.c_out
        out[c.name] = (w, gam, bet)
    nh = ch * base * 9
    out["head"] = (theta[o:o + nh].reshape(ch, base, 3, 3), theta[o + nh:o + nh + ch])
    assert o + nh + ch == theta.numel()
    return out


def init_params(levels: int, base: int, seed: int = 0, ch: int = 1) -> np.ndarray:
    """He-normal convolution weights, gamma 1, beta 0, head bias 0 (float32)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for c in conv_list(levels, base, ch):
        std = math.sqrt(2.0 / (9 * c.c_in))
        parts += [rng.normal(0.0, std, c.c_out * c.c_in * 9), np.ones(c.c_out), np.zeros(c.c_out)]
    parts += [rng.normal(0.0, math.sqrt(1.0 / (9 * base)), ch * base * 9), np.zeros(ch)]
    return np.concatenate(parts).astype(np.float32)


def bf16(x, on: bool = True):
    """Round to bfloat16 (nearest, ties to even) as the stored value, with an
    identity derivative (the rounding is a storage format, not part of the
    function being differentiated)."""
    if not on:
        return x
    return x + (x.to(torch.bfloat16).to(x.dtype) - x).detach()


def conv_bn_relu(x, w, gamma, beta, eps, quant: bool = False):
    """3x3 convolution (padding 1, no bias), BatchNorm on batch statistics, ReLU.
    With quant, the conv output z and the activation are stored in bfloat16 and
    the statistics are those of the stored z."""
    z = bf16(F.conv2d(x, bf16(w, quant), padding=1), quant)
    y = F.batch_norm(z, None, None, gamma, beta, training=True, eps=eps)
    return z, bf16(F.relu(y), quant)


def up2(x):
    """Bilinear x2 upsampling, half-pixel centres (align_corners=False)."""
    return F.interpolate(x, scale_factor=2, mode="bilinear", align_corners=False)


def _as_channels(x, ch: int):
    """[I, n, n] scans for one channel, [I, ch, n, n] otherwise -> [I, ch, n, n]."""
    return x[:, None] if ch == 1 else x


def _from_channels(m, ch: int):
    return m[:, 0] if ch == 1 else m


def forward(x, theta, levels: int, base: int, eps: float = 1e-5, keep: bool = False,
            quant: bool = False, ch: int = 1):
    """Masks for images x [I, n, n] (ch = 1) or [I, ch, n, n] (FP64 tensors); theta is
    the flat FP64 vector.  Returns m of the same shape as x and, with keep=True, every
    intermediate by name.  quant=True stores the scan, the conv weights, every conv
    output, activation and upsampled tensor in bfloat16 (the arithmetic stays FP64);
    the head's weights and everything after the last activation stay unrounded."""
    P = unpack(theta, levels, base, ch)
    h = bf16(_as_channels(x, ch), quant)
    acts, skips = {}, []
    for l in range(levels):
        if l > 0:
            h = F.max_pool2d(h, 2)
            acts[f"pool{l}"] = h
        for part in "ab":
            z, h = conv_bn_relu(h, *P[f"enc{l}{part}"], eps, quant)
            acts[f"enc{l}{part}.z"], acts[f"enc{l}{part}"] = z, h
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        h = torch.cat([bf16(up2(h), quant), skips[l]], dim=1)
        acts[f"cat{l}"] = h
        for part in "ab":
            z, h = conv_bn_relu(h, *P[f"dec{l}{part}"], eps, quant)
            acts[f"dec{l}{part}.z"], acts[f"dec{l}{part}"] = z, h
    wh, bh = P["head"]
    logit = F.conv2d(h, wh, bh, padding=1)
    m = _from_channels(torch.sigmoid(logit), ch)
    acts["logit"] = _from_channels(logit, ch)
    return (m, acts) if keep else m


def batch_stats(z):
    """Per-channel batch mean and biased variance of a conv output [I, C, H, W]."""
    return z.mean(dim=(0, 2, 3)), z.var(dim=(0, 2, 3), unbiased=False)


def pose_loss(pose, target, kind: str):
    """Eq. 13 averaged over the batch: L1 (the paper) or L2 (squared) of
    (theta, t_x, t_y) with theta in rad and t in m, unweighted."""
    d = pose - target
    if kind == "l1":
        return d.abs().sum(dim=1).mean()
    if kind == "l2":
        return (d * d).sum(dim=1).mean()
    raise ValueError(kind)


def adam_step(theta, grad, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999,
              eps: float = 1e-8):
    """One Adam update (bias-corrected moments); returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (torch.sqrt(vh) + eps), m, v


def running_stats(x, theta, levels: int, base: int, run_mean, run_var, momentum: float = 0.1,
                  eps: float = 1e-5, quant: bool = False, ch: int = 1):
    """Running statistics after one training pass: each BN channel moves by
    `momentum` towards its batch mean and unbiased batch variance."""
    _, acts = forward(x, theta, levels, base, eps, keep=True, quant=quant, ch=ch)
    means, vars_ = [], []
    for c in conv_list(levels, base, ch):
        z = acts[f"{c.name}.z"]
        means.append(z.mean(dim=(0, 2, 3)))
        vars_.append(z.var(dim=(0, 2, 3), unbiased=True))
    mu, var = torch.cat(means), torch.cat(vars_)
    return (1 - momentum) * run_mean + momentum * mu, (1 - momentum) * run_var + momentum * var


def forward_eval(x, theta, levels: int, base: int, run_mean, run_var, eps: float = 1e-5, ch: int = 1,
                 quant: bool = False):
    """Masks with BatchNorm on the given running statistics (inference).
    quant=True stores in bfloat16 what the training forward's quant mode
    stores (the scan, the conv weights, every conv output, activation and
    upsampled tensor); the arithmetic stays FP64."""
    P = unpack(theta, levels, base, ch)
    stats, o = {}, 0
    for c in conv_list(levels, base, ch):
        stats[c.name] = (run_mean[o:o + c.c_out], run_var[o:o + c.c_out])
        o += c.c_out

    def cbr(h, name):
        w, g, b = P[name]
        z = bf16(F.conv2d(h, bf16(w, quant), padding=1), quant)
        return bf16(F.relu(F.batch_norm(z, *stats[name], g, b, training=False, eps=eps)), quant)

    h, skips = bf16(_as_channels(x, ch), quant), []
    for l in range(levels):
        if l > 0:
            h = F.max_pool2d(h, 2)
        h = cbr(cbr(h, f"enc{l}a"), f"enc{l}b")
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        h = torch.cat([bf16(up2(h), quant), skips[l]], dim=1)
        h = cbr(cbr(h, f"dec{l}a"), f"dec{l}b")
    wh, bh = P["head"]
    return _from_channels(torch.sigmoid(F.conv2d(h, wh, bh, padding=1)), ch)


def grad(x, d_mask, theta, levels: int, base: int, eps: float = 1e-5, quant: bool = False, ch: int = 1):
    """d<mask, d_mask>/d theta by FP64 autograd (the mask network's adjoint)."""
    th = theta.detach().clone().requires_grad_(True)
    m = forward(x, th, levels, base, eps, quant=quant, ch=ch)
    (m * d_mask).sum().backward()
    return th.grad.detach()


def grad_input(x, d_mask, theta, levels: int, base: int, eps: float = 1e-5, quant: bool = False,
               ch: int = 1):
    """d<mask, d_mask>/d x, the gradient with respect to the input scans, by FP64 autograd
    (through the training forward's batch statistics, like ``grad``)."""
    xx = torch.as_tensor(x).to(torch.float64).detach().clone().requires_grad_(True)
    m = forward(xx, theta.detach(), levels, base, eps, quant=quant, ch=ch)
    (m * d_mask).sum().backward()
    return xx.grad.detach()
