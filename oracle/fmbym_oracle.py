"""FP64 CPU oracle of the decoupled correlative pose search (Fast-MbyM).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path imports this module:
only the tests, the smoke check and the benchmark's CPU-baseline leg use it.
It shares no code with the HIP library and imports nothing from the package.

Everything is plain, slow and written to be read against the paper:
  * every transform is a naive DFT written as a product with the matrix
    W_n[k, m] = exp(-2 pi i ((k m) mod n) / n) (no FFT library);
  * bilinear resampling is explicit floor / weight arithmetic;
  * correlations are their defining sums where that is affordable, and the
    cross-correlation theorem with naive DFTs otherwise (the equivalence is
    itself pinned by the tests);
  * gradients come from torch autograd over this same FP64 code.

Conventions.  Scans are [n, n] arrays; row i is y = (i - c) delta and column
j is x = (j - c) delta with the origin pixel c = floor(n/2) (n/2 for the even
sizes, (n - 1)/2 for the odd sizes the paper measures); the sensor is pixel
(c, c).  R(theta) rotates x toward y.  The pose satisfies Eq. 1,
f(x) ~= g(R x + t).  Forward DFTs are unnormalised, inverse DFTs carry 1/n
per axis.

Readings of passages that the paper leaves open (all shared with the HIP
library, which implements the same definitions):
  * Correlation keeps the conjugate of Eq. 3 (Algorithm 1 writes the two
    correlations as products of FFTs without one, which would be a
    convolution and returns -theta).
  * The angle score is Eq. 8's zero-radial-offset slice: a circular
    correlation along angle per radius, averaged over radius (Algorithm 1's
    "Mean over r").  The marginal reading is available as ``angle_marginal``.
  * Candidate grids are the lag grids theta_l = l pi / n_theta and
    t' = s delta with l, s in [-floor(n/2), n - 1 - floor(n/2)] (Algorithm 1's
    Linspace lists): [-n/2, n/2) for even n, symmetric for odd n.
  * The Hann window is the periodic one, applied as an outer product; stage 2
    uses the windowed scans (Algorithm 1 reassigns f and g).  Written about the
    origin pixel, h[k] = (1 + cos(2 pi (k - c) / n)) / 2, which is the periodic
    Hann for even n and its symmetric counterpart about c for odd n.
  * The band-pass is a hard annulus band_lo <= |k|/n <= band_hi in cycles per
    pixel (disabled when band_hi <= 0).
  * Polar grid: n_theta angles over [0, pi) and n_r radii over [0, n/2) bins;
    bilinear on the lattice with indices taken modulo n.
  * Rotate samples g at R(theta) y about the origin pixel with zeros outside.
  * ZeroPad pads to 2n, so c_xy is the exact linear correlation for every lag
    of the window (the lag grid above, on both axes).
  * The frame change is t = R(theta) t' (Eq. 1 together with the conventions
    above; Algorithm 1's BuildSO2(-theta) matches the reversed correlation
    order).
  * Soft-argmax uses softmax((c - max c) / T); with ``zscore`` the scores are
    first standardised (c - mean) / std.  With ``hard_argmax`` both stages take
    the lag of the first maximum instead (the search of Eq. 2-3 without the
    soft relaxation).
"""
from __future__ import annotations

import dataclasses
import math

import torch

F64 = torch.float64
C128 = torch.complex128


@dataclasses.dataclass(frozen=True)
class Params:
    """ScanMatch's parameters (Algorithm 1) plus the readings listed above."""

    n: int
    n_theta: int
    n_r: int | None = None          # polar radii; the method uses n (Section III-D)
    delta_xy: float = 1.0           # metres per pixel
    temp_theta: float = 1.0
    temp_xy: float = 1.0
    band_lo: float = 0.0            # cycles per pixel
    band_hi: float = 0.0            # <= 0 disables the band-pass
    hann: bool = True
    angle_marginal: bool = False
    zscore: bool = False
    xy_unwindowed: bool = False
    hard_argmax: bool = False

    @property
    def radii(self) -> int:
        return self.n if self.n_r is None else self.n_r


# ---------------------------------------------------------------- transforms

def dft_matrix(n: int) -> torch.Tensor:
    """W[k, m] = exp(-2 pi i ((k m) mod n) / n), the n-point forward DFT (Eq. 14)."""
    k = torch.arange(n, dtype=torch.int64)
    km = (k[:, None] * k[None, :]) % n
    ang = (-2.0 * math.pi / n) * km.to(F64)
    return torch.complex(torch.cos(ang), torch.sin(ang))


def dft2(x: torch.Tensor) -> torch.Tensor:
    """2-D DFT over the last two axes: F = W_rows x W_cols^T (Algorithm 1, FFT2d)."""
    r, c = x.shape[-2], x.shape[-1]
    return dft_matrix(r) @ x.to(C128) @ dft_matrix(c).transpose(0, 1)


def idft2(x: torch.Tensor) -> torch.Tensor:
    """Inverse 2-D DFT with 1/(rows cols) (Algorithm 1, iFFT2d)."""
    r, c = x.shape[-2], x.shape[-1]
    wr = dft_matrix(r).conj()
    wc = dft_matrix(c).conj()
    return (wr @ x.to(C128) @ wc.transpose(0, 1)) / (r * c)


def dft1(x: torch.Tensor) -> torch.Tensor:
    """1-D DFT along the last axis."""
    return x.to(C128) @ dft_matrix(x.shape[-1]).transpose(0, 1)


def idft1(x: torch.Tensor) -> torch.Tensor:
    n = x.shape[-1]
    return (x.to(C128) @ dft_matrix(n).conj().transpose(0, 1)) / n


# ------------------------------------------------------------------- filters

def hann_periodic(n: int) -> torch.Tensor:
    """h[k] = (1 - cos(2 pi k / n)) / 2 (Algorithm 1, HanningFilter)."""
    k = torch.arange(n, dtype=F64)
    return 0.5 * (1.0 - torch.cos(2.0 * math.pi * k / n))


def hann_centred(n: int) -> torch.Tensor:
    """h[k] = (1 + cos(2 pi (k - c) / n)) / 2 about the origin pixel c = floor(n/2):
    the periodic Hann for even n, peaked at and symmetric about c for odd n."""
    k = torch.arange(n, dtype=F64) - (n // 2)
    return 0.5 * (1.0 + torch.cos(2.0 * math.pi * k / n))


def hann2d(n: int) -> torch.Tensor:
    h = hann_centred(n)
    return h[:, None] * h[None, :]


def signed_freq(n: int) -> torch.Tensor:
    """Frequency index of DFT bin k, mapped to [-n/2, n/2) (odd n: [-(n-1)/2, (n-1)/2])."""
    k = torch.arange(n, dtype=torch.int64)
    return torch.where(k < (n + 1) // 2, k, k - n) if n % 2 else torch.where(k < n // 2, k, k - n)


def band_mask(n: int, lo: float, hi: float) -> torch.Tensor:
    """Hard radial annulus lo <= |k|/n <= hi in cycles per pixel (Algorithm 1, BandPassFilter)."""
    if hi <= 0.0:
        return torch.ones(n, n, dtype=F64)
    k = signed_freq(n).to(F64)
    rho = torch.sqrt(k[:, None] ** 2 + k[None, :] ** 2) / n
    return ((rho >= lo) & (rho <= hi)).to(F64)


# ---------------------------------------------------------------- resampling

def bilinear_periodic(a: torch.Tensor, row: torch.Tensor, col: torch.Tensor) -> torch.Tensor:
    """Bilinear sample of a[..., n, n] at fractional (row, col), indices modulo n."""
    n0, n1 = a.shape[-2], a.shape[-1]
    r0 = torch.floor(row)
    c0 = torch.floor(col)
    wr = row - r0
    wc = col - c0
    r0 = r0.to(torch.int64)
    c0 = c0.to(torch.int64)
    out = 0.0
    for dr, wgt_r in ((0, 1.0 - wr), (1, wr)):
        for dc, wgt_c in ((0, 1.0 - wc), (1, wc)):
            out = out + wgt_r * wgt_c * a[..., (r0 + dr) % n0, (c0 + dc) % n1]
    return out


def bilinear_zero(a: torch.Tensor, row: torch.Tensor, col: torch.Tensor) -> torch.Tensor:
    """Bilinear sample of a[n, n] at fractional (row, col); lattice points outside read as zero."""
    n0, n1 = a.shape[-2], a.shape[-1]
    r0 = torch.floor(row)
    c0 = torch.floor(col)
    wr = row - r0
    wc = col - c0
    r0 = r0.to(torch.int64)
    c0 = c0.to(torch.int64)
    out = 0.0
    for dr, wgt_r in ((0, 1.0 - wr), (1, wr)):
        for dc, wgt_c in ((0, 1.0 - wc), (1, wc)):
            rr = r0 + dr
            cc = c0 + dc
            inside = (rr >= 0) & (rr < n0) & (cc >= 0) & (cc < n1)
            v = a[rr.clamp(0, n0 - 1), cc.clamp(0, n1 - 1)]
            out = out + wgt_r * wgt_c * torch.where(inside, v, torch.zeros_like(v))
    return out


def polar_grid(n: int, n_r: int, n_theta: int):
    """Sample coordinates (row, col) of the polar grid: angle pi a / n_theta, radius (n/2) b / n_r."""
    phi = math.pi * torch.arange(n_theta, dtype=F64) / n_theta
    rho = (n / 2.0) * torch.arange(n_r, dtype=F64) / n_r
    u_x = rho[:, None] * torch.cos(phi)[None, :]
    u_y = rho[:, None] * torch.sin(phi)[None, :]
    return u_y, u_x


def cart2pol(a: torch.Tensor, n_r: int, n_theta: int) -> torch.Tensor:
    """Polar resampling of a magnitude spectrum, [n, n] -> [n_r, n_theta] (Algorithm 1, Cart2Pol).

    Frequency (u_x, u_y) = rho (cos phi, sin phi) is read from DFT bin
    (row u_y mod n, column u_x mod n), the periodic extension of the DFT.
    """
    u_y, u_x = polar_grid(a.shape[-1], n_r, n_theta)
    return bilinear_periodic(a, u_y, u_x)


def rotate(g: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """g'(y) = g(R(theta) y) about the origin pixel floor(n/2), bilinear, zeros outside
    (Algorithm 1, Rotate)."""
    n = g.shape[-1]
    o = n // 2
    c = torch.arange(n, dtype=F64) - o
    yx = c[None, :].expand(n, n)            # x offset of output pixel [i, j]
    yy = c[:, None].expand(n, n)            # y offset
    ct, st = torch.cos(theta), torch.sin(theta)
    px = ct * yx - st * yy
    py = st * yx + ct * yy
    return bilinear_zero(g, py + o, px + o)


# -------------------------------------------------------------- correlations

def lag_indices(n: int) -> torch.Tensor:
    """Lags -floor(n/2) .. n - 1 - floor(n/2) in storage order ([-n/2, n/2) for even n)."""
    return torch.arange(n, dtype=torch.int64) - n // 2


def angle_correlation(pf: torch.Tensor, pg: torch.Tensor) -> torch.Tensor:
    """c[l] = (1/n_r) sum_b sum_a pf[b, a] pg[b, (a + l) mod n_theta] for l on the lag grid (Eq. 8).

    The defining sum, evaluated one lag at a time (wrap padding along angle).
    """
    n_r, n_t = pf.shape
    out = []
    for l in lag_indices(n_t).tolist():
        out.append((pf * torch.roll(pg, shifts=-l, dims=1)).sum())
    return torch.stack(out) / n_r


def angle_correlation_marginal(pf: torch.Tensor, pg: torch.Tensor) -> torch.Tensor:
    """Reading 'Mean over r of the 2-D correlation': the circular correlation of radius-summed profiles."""
    n_r = pf.shape[0]
    return angle_correlation(pf.sum(0, keepdim=True), pg.sum(0, keepdim=True)) / n_r


def xy_correlation_direct(fw: torch.Tensor, gp: torch.Tensor) -> torch.Tensor:
    """c[s] = sum_x fw[x] gp[x + s], linear (zero outside), s on the lag grid squared (Eq. 3 on
    the lattice).  Storage [i, j] holds lag (s_y, s_x) = (i - floor(n/2), j - floor(n/2)).
    O(n^4): tiny n only.
    """
    n = fw.shape[-1]
    lags = lag_indices(n).tolist()
    rows = []
    for sy in lags:
        row = []
        for sx in lags:
            y0, y1 = max(0, -sy), min(n, n - sy)
            x0, x1 = max(0, -sx), min(n, n - sx)
            row.append((fw[y0:y1, x0:x1] * gp[y0 + sy:y1 + sy, x0 + sx:x1 + sx]).sum())
        rows.append(torch.stack(row))
    return torch.stack(rows)


def xy_correlation(fw: torch.Tensor, gp: torch.Tensor) -> torch.Tensor:
    """Same as ``xy_correlation_direct`` through ZeroPad to 2n and the cross-correlation theorem.

    c = iDFT2(conj(DFT2(pad fw)) * DFT2(pad gp)), read at lags s mod 2n.
    """
    n = fw.shape[-1]
    m = 2 * n
    pf = torch.nn.functional.pad(fw, (0, n, 0, n))
    pg = torch.nn.functional.pad(gp, (0, n, 0, n))
    c = idft2(dft2(pf).conj() * dft2(pg)).real
    idx = lag_indices(n) % m
    return c[idx[:, None], idx[None, :]]


# --------------------------------------------------------------- soft-argmax

def argmax_weights(c: torch.Tensor) -> torch.Tensor:
    """One-hot weights at the first maximum of c in storage (row-major) order."""
    w = torch.zeros(c.numel(), dtype=c.dtype)
    w[int(torch.argmax(c.reshape(-1)))] = 1.0
    return w.reshape(c.shape)


def score_weights(c: torch.Tensor, p: "Params", temp: float) -> torch.Tensor:
    """The weights of a stage's candidates: hard argmax or temperature softmax."""
    return argmax_weights(c) if p.hard_argmax else softmax_weights(c, temp, p.zscore)


def softmax_weights(c: torch.Tensor, temp: float, zscore: bool) -> torch.Tensor:
    """p = softmax((c - max c) / T) over all entries (Section III-D, SoftArgMax)."""
    z = c.reshape(-1)
    if zscore:
        z = (z - z.mean()) / z.std(unbiased=False)
    z = (z - z.max()) / temp
    e = torch.exp(z)
    return (e / e.sum()).reshape(c.shape)


# -------------------------------------------------------------------- search

def stage_rotation(fw: torch.Tensor, gw: torch.Tensor, p: Params):
    """Stage 1 of Algorithm 1: heading from polar magnitude spectra (Eq. 5-8)."""
    band = band_mask(p.n, p.band_lo, p.band_hi)
    af = band * torch.abs(dft2(fw))
    ag = band * torch.abs(dft2(gw))
    pf = cart2pol(af, p.radii, p.n_theta)
    pg = cart2pol(ag, p.radii, p.n_theta)
    c_theta = angle_correlation_marginal(pf, pg) if p.angle_marginal else angle_correlation(pf, pg)
    grid = lag_indices(p.n_theta).to(F64) * (math.pi / p.n_theta)
    w = score_weights(c_theta, p, p.temp_theta)
    theta = (w * grid).sum()
    return theta, c_theta, dict(af=af, ag=ag, pf=pf, pg=pg)


def stage_translation(fw: torch.Tensor, gw: torch.Tensor, theta: torch.Tensor, p: Params,
                      direct: bool = False):
    """Stage 2 of Algorithm 1: translation from the correlation with g rotated by theta (Eq. 9)."""
    gp = rotate(gw, theta)
    c_xy = xy_correlation_direct(fw, gp) if direct else xy_correlation(fw, gp)
    lag = lag_indices(p.n).to(F64) * p.delta_xy
    w = score_weights(c_xy, p, p.temp_xy)
    tpx = (w * lag[None, :]).sum()
    tpy = (w * lag[:, None]).sum()
    ct, st = torch.cos(theta), torch.sin(theta)
    tx = ct * tpx - st * tpy
    ty = st * tpx + ct * tpy
    return tx, ty, c_xy, dict(gp=gp, tp=(tpx, tpy))


def search(f, g, p: Params, m_f=None, m_g=None, direct: bool = False) -> dict:
    """ScanMatch (Algorithm 1) on masked scans (Eq. 11-12): returns pose and both score surfaces.

    ``f``, ``g`` (and masks) are [n, n]; anything array-like is upcast to FP64.
    Gradients flow to any input that requires them.
    """
    f = torch.as_tensor(f).to(F64)
    g = torch.as_tensor(g).to(F64)
    if m_f is not None:
        f = f * torch.as_tensor(m_f).to(F64)
    if m_g is not None:
        g = g * torch.as_tensor(m_g).to(F64)
    if p.hann:
        w = hann2d(p.n)
        fw, gw = w * f, w * g
    else:
        fw, gw = f, g
    theta, c_theta, aux1 = stage_rotation(fw, gw, p)
    if p.xy_unwindowed:
        tx, ty, c_xy, aux2 = stage_translation(f, g, theta, p, direct)
    else:
        tx, ty, c_xy, aux2 = stage_translation(fw, gw, theta, p, direct)
    return dict(theta=theta, tx=tx, ty=ty, pose=torch.stack([theta, tx, ty]),
                c_theta=c_theta, c_xy=c_xy, fw=fw, gw=gw, **aux1, **aux2)


def search_batch(f, g, p: Params, m_f=None, m_g=None) -> dict:
    """``search`` over a leading batch axis; returns stacked pose [B, 3], c_theta, c_xy."""
    outs = []
    for b in range(len(f)):
        outs.append(search(f[b], g[b], p, None if m_f is None else m_f[b],
                           None if m_g is None else m_g[b]))
    return dict(pose=torch.stack([o["pose"] for o in outs]),
                c_theta=torch.stack([o["c_theta"] for o in outs]),
                c_xy=torch.stack([o["c_xy"] for o in outs]))


def search_grad(f, g, d_pose, p: Params, m_f=None, m_g=None) -> dict:
    """FP64 autograd of <d_pose, pose(f, g, m_f, m_g)>; absent masks give no mask gradient."""
    f = torch.as_tensor(f).to(F64).clone().requires_grad_(True)
    g = torch.as_tensor(g).to(F64).clone().requires_grad_(True)
    mf = None if m_f is None else torch.as_tensor(m_f).to(F64).clone().requires_grad_(True)
    mg = None if m_g is None else torch.as_tensor(m_g).to(F64).clone().requires_grad_(True)
    out = search(f, g, p, mf, mg)
    (out["pose"] * torch.as_tensor(d_pose).to(F64)).sum().backward()
    res = dict(d_f=f.grad, d_g=g.grad, pose=out["pose"].detach())
    if mf is not None:
        res["d_m_f"] = mf.grad
        res["d_m_g"] = mg.grad
    return res


# ------------------------------------------ full-circle heading (Conclusion)

def search_full_circle(f, g, p: Params, m_f=None, m_g=None) -> dict:
    """Heading over the whole circle, for the metric localisation with arbitrary
    rotational offset that the Conclusion proposes.

    Stage 1 sees only magnitude spectra, and those of real scans are point
    symmetric (|F(-k)| = |F(k)|, the property behind Eq. 5-6), so it fixes the
    heading modulo pi.  Headings theta and theta + pi give different rotated
    scans, though, so stage 2 (Eq. 9) tells them apart: run it at both and
    keep the one whose correlation surface has the larger peak (max over the
    lags of c_xy; the stage-1 heading on ties).  The other heading is written
    in [-pi, pi): theta + pi for theta < 0, else theta - pi.  Its pose is
    that stage's own soft-argmax translation, t = R(theta + pi) t'.
    """
    out = search(f, g, p, m_f, m_g)
    theta = out["theta"]
    alt = theta + math.pi if float(theta) < 0 else theta - math.pi
    if p.xy_unwindowed:
        f2 = torch.as_tensor(f).to(F64)
        g2 = torch.as_tensor(g).to(F64)
        if m_f is not None:
            f2 = f2 * torch.as_tensor(m_f).to(F64)
        if m_g is not None:
            g2 = g2 * torch.as_tensor(m_g).to(F64)
    else:
        f2, g2 = out["fw"], out["gw"]
    tx2, ty2, c_xy2, _ = stage_translation(f2, g2, alt, p)
    peaks = torch.stack([out["c_xy"].max(), c_xy2.max()])
    turned = bool(peaks[1] > peaks[0])
    pose = torch.stack([alt, tx2, ty2]) if turned else out["pose"]
    return dict(pose=pose, peaks=peaks, turned=turned, plain=out["pose"], c_xy_turned=c_xy2)


# ------------------------------------------------- plain joint search (Eq. 2)

def joint_headings(n_angles: int) -> torch.Tensor:
    """Candidate headings of the joint comparator: -pi/2 + k pi / n_angles, k < n_angles
    (the range of the decoupled search's lag grid, R3, at a coarser step)."""
    return -math.pi / 2 + torch.arange(n_angles, dtype=F64) * (math.pi / n_angles)


def joint_search_rotated(f, g, p: Params, thetas, m_f=None, m_g=None) -> dict:
    """Brute-force joint search on the translation stage's lag grid (Eq. 2-3 with
    the search over headings done exhaustively instead of by Eq. 8).

    For every candidate heading theta_k, the stage-2 correlation at that fixed
    heading, J_k(s') = sum_x fw(x) Rotate(gw, theta_k)(x + s') (Eq. 9); the pose
    is the hard argmax over (k, s') with t = R(theta_k) s' delta (R9), first
    maximum in (k, s_y, s_x) order.  J_k(s') = S_k(R(theta_k) s') in the
    notation of ``joint_scores``.
    """
    f = torch.as_tensor(f).to(F64)
    g = torch.as_tensor(g).to(F64)
    if m_f is not None:
        f = f * torch.as_tensor(m_f).to(F64)
    if m_g is not None:
        g = g * torch.as_tensor(m_g).to(F64)
    w = hann2d(p.n) if p.hann else torch.ones(p.n, p.n, dtype=F64)
    fw, gw = (f, g) if p.xy_unwindowed else (w * f, w * g)
    thetas = torch.as_tensor(thetas).to(F64)
    scores = torch.stack([xy_correlation(fw, rotate(gw, th)) for th in thetas])
    flat = int(torch.argmax(scores.reshape(-1)))
    k, rem = divmod(flat, p.n * p.n)
    iy, ix = divmod(rem, p.n)
    th = thetas[k]
    tpx, tpy = (ix - p.n // 2) * p.delta_xy, (iy - p.n // 2) * p.delta_xy
    ct, st = math.cos(float(th)), math.sin(float(th))
    return dict(scores=scores, peak=scores.reshape(len(thetas), -1).max(dim=1).values, theta=float(th),
                tx=ct * tpx - st * tpy, ty=st * tpx + ct * tpy, index=(k, iy, ix),
                pose=torch.tensor([float(th), ct * tpx - st * tpy, st * tpx + ct * tpy], dtype=F64))


def joint_scores(fw: torch.Tensor, gw: torch.Tensor, thetas, n_lag: int) -> torch.Tensor:
    """S[k, s_y, s_x] = sum_x fw(x) g(R(theta_k) x + s), the correlative search of Eq. 2-3.

    g is sampled bilinearly with zeros outside; s runs over the integer lags
    [-n_lag/2, n_lag/2)^2 in pixels.  Direct sums: tiny n only.
    """
    n = fw.shape[-1]
    o = n // 2
    c = torch.arange(n, dtype=F64) - o
    xx = c[None, :].expand(n, n)
    yy = c[:, None].expand(n, n)
    lags = lag_indices(n_lag).tolist()
    out = torch.zeros(len(thetas), n_lag, n_lag, dtype=F64)
    for k, th in enumerate(thetas):
        ct, st = math.cos(th), math.sin(th)
        px = ct * xx - st * yy
        py = st * xx + ct * yy
        for iy, sy in enumerate(lags):
            for ix, sx in enumerate(lags):
                v = bilinear_zero(gw, py + sy + o, px + sx + o)
                out[k, iy, ix] = (fw * v).sum()
    return out


def joint_search(f, g, p: Params, thetas, n_lag: int | None = None) -> dict:
    """Brute-force joint argmax over (theta_k, s); the comparison the decoupling approximates."""
    f = torch.as_tensor(f).to(F64)
    g = torch.as_tensor(g).to(F64)
    w = hann2d(p.n) if p.hann else torch.ones(p.n, p.n, dtype=F64)
    n_lag = p.n if n_lag is None else n_lag
    s = joint_scores(w * f, w * g, thetas, n_lag)
    k, iy, ix = [int(v) for v in torch.unravel_index(torch.argmax(s), s.shape)]
    # S peaks where g(R x + s) matches f(x), so s is Eq. 1's t directly (no frame change)
    return dict(scores=s, theta=float(thetas[k]), tx=(ix - n_lag // 2) * p.delta_xy,
                ty=(iy - n_lag // 2) * p.delta_xy, index=(k, iy, ix))
