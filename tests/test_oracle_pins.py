"""Pins of the FP64 oracle against what the paper and the mathematics fix.

None of these retypes an oracle formula: each compares the oracle with an
independent fact (a library transform, a pure-Python defining sum, an exact
symmetry of the Fourier transform, a closed form, a brute-force search, or
finite differences), chosen so that a dropped term, a wrong sign or index, or
a transposed operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import synth

F64 = torch.float64


def rnd(*shape, seed=0):
    return torch.as_tensor(np.random.default_rng(seed).standard_normal(shape), dtype=F64)


# ----------------------------------------------------------------- transforms

def test_dft_is_the_library_fft():
    """The naive DFT-matrix transform equals numpy's FFT (forward unnormalised, inverse 1/n)."""
    x = rnd(12, 16) + 1j * rnd(12, 16, seed=1)
    np.testing.assert_allclose(O.dft2(x).numpy(), np.fft.fft2(x.numpy()), atol=1e-11)
    np.testing.assert_allclose(O.idft2(x).numpy(), np.fft.ifft2(x.numpy()), atol=1e-13)
    np.testing.assert_allclose(O.dft1(x).numpy(), np.fft.fft(x.numpy(), axis=-1), atol=1e-11)
    np.testing.assert_allclose(O.idft1(x).numpy(), np.fft.ifft(x.numpy(), axis=-1), atol=1e-13)


def test_parseval():
    """sum |f|^2 = (1/(n m)) sum |F|^2 pins the DFT normalisation."""
    f = rnd(16, 16, seed=3)
    F = O.dft2(f)
    assert abs(float((f ** 2).sum()) - float((F.abs() ** 2).sum()) / 256) < 1e-10


def test_magnitude_spectrum_ignores_circular_shifts():
    """Eq. 5-7: translating a scan changes only the phase of its spectrum."""
    f = rnd(16, 16, seed=4)
    for s in [(3, -5), (0, 7), (-8, 1)]:
        g = torch.roll(f, shifts=s, dims=(0, 1))
        np.testing.assert_allclose(O.dft2(g).abs().numpy(), O.dft2(f).abs().numpy(), atol=1e-11)


def _quarter_turn(f):
    """g with g(R(90 deg) x) = f(x) on the circular lattice: g[j, (n - i) mod n] = f[i, j]."""
    n = f.shape[0]
    g = torch.empty_like(f)
    for i in range(n):
        for j in range(n):
            g[j, (n - i) % n] = f[i, j]
    return g


def test_magnitude_spectrum_rotates_with_the_scan():
    """Eq. 7: |F|(u) = |G|(R u).  Exact for a lattice quarter turn: bin (ky, kx) -> (kx, -ky)."""
    n = 12
    f = rnd(n, n, seed=5)
    g = _quarter_turn(f)
    af, ag = O.dft2(f).abs(), O.dft2(g).abs()
    for ky in range(n):
        for kx in range(n):
            assert abs(float(af[ky, kx]) - float(ag[kx, (-ky) % n])) < 1e-10


def test_polar_resampling_orientation():
    """Bilinear reproduces linear functions: a column ramp reads rho cos(phi), a row ramp rho sin(phi).

    A transposed operand or a wrong angle direction in Cart2Pol fails here.
    """
    n, n_r, n_t = 64, 16, 24
    k = torch.arange(n, dtype=F64)
    ramp_x = k[None, :].expand(n, n).clone()    # value = column index
    ramp_y = k[:, None].expand(n, n).clone()    # value = row index
    # keep away from the modular wrap: shift the ramps so the read region is interior
    # (polar radii span [0, n/4) when n_r samples cover n/2 bins -> use n_r = n/4 * ...)
    rho = (n / 2.0) * torch.arange(n_r, dtype=F64) / n_r
    phi = math.pi * torch.arange(n_t, dtype=F64) / n_t
    pol_x = O.cart2pol(torch.roll(ramp_x, shifts=n // 2, dims=1) - n // 2, n_r, n_t)
    pol_y = O.cart2pol(torch.roll(ramp_y, shifts=n // 2, dims=0) - n // 2, n_r, n_t)
    # rolled ramps hold the signed index k - n/2 at bin (k + n/2) mod n, i.e. value == signed bin
    # coordinate for |coordinate| < n/2
    np.testing.assert_allclose(pol_x.numpy(), (rho[:, None] * torch.cos(phi)[None, :]).numpy(), atol=1e-9)
    np.testing.assert_allclose(pol_y.numpy(), (rho[:, None] * torch.sin(phi)[None, :]).numpy(), atol=1e-9)


def test_polar_spectra_of_a_quarter_turn_are_shifted_by_half_the_angle_axis():
    """Stage 1 end to end on an exact rotation: polar magnitudes shift by n_theta/2 bins (pi/2)."""
    n, n_t = 16, 8
    f = rnd(n, n, seed=6)
    g = _quarter_turn(f)
    pf = O.cart2pol(O.dft2(f).abs(), n, n_t)
    pg = O.cart2pol(O.dft2(g).abs(), n, n_t)
    np.testing.assert_allclose(pf.numpy(), torch.roll(pg, shifts=-n_t // 2, dims=1).numpy(), atol=1e-9)
    c = O.angle_correlation(pf, pg)
    assert int(torch.argmax(c)) == 0   # lag -n/2, i.e. -pi/2 == +pi/2 modulo pi


def test_rotate_direction_and_linear_exactness():
    """Rotate samples g at R(theta) y: a linear ramp g = x comes back as cos(th) x - sin(th) y."""
    n = 32
    c = torch.arange(n, dtype=F64) - n / 2
    xs = c[None, :].expand(n, n).clone()
    ys = c[:, None].expand(n, n).clone()
    th = torch.tensor(0.3, dtype=F64)
    out = O.rotate(xs, th)
    want = math.cos(0.3) * xs - math.sin(0.3) * ys
    # interior: sample position and its bilinear cell inside the grid
    px = math.cos(0.3) * xs - math.sin(0.3) * ys + n / 2
    py = math.sin(0.3) * xs + math.cos(0.3) * ys + n / 2
    inside = (px >= 0) & (px < n - 1) & (py >= 0) & (py < n - 1)
    np.testing.assert_allclose(out[inside].numpy(), want[inside].numpy(), atol=1e-10)
    # a quarter turn is a permutation of the lattice: g'(y) = g(R y)
    g = rnd(n, n, seed=7)
    gq = O.rotate(g, torch.tensor(math.pi / 2, dtype=F64))
    for i in range(1, n):
        for j in range(1, n):
            # y = (j - n/2, i - n/2) -> R y = (-(i - n/2), j - n/2) -> column n - i, row j
            assert abs(float(gq[i, j]) - float(g[j, n - i])) < 1e-12


def test_hann_window_values():
    """Periodic Hann: h[0] = 0, h[n/4] = 1/2, h[n/2] = 1, sum = n/2."""
    h = O.hann_periodic(32)
    assert float(h[0]) == 0.0 and abs(float(h[16]) - 1.0) < 1e-15 and abs(float(h[8]) - 0.5) < 1e-15
    assert abs(float(h.sum()) - 16.0) < 1e-12
    w = O.hann2d(32)
    assert float(w[16, 16]) == pytest.approx(1.0) and float(w[0, 5]) == 0.0


def test_band_mask_annulus():
    """Band-pass keeps |k|/n in [lo, hi]: DC and the far corner are cut, a mid ring is kept."""
    n = 64
    b = O.band_mask(n, 0.02, 0.4)
    assert b[0, 0] == 0 and b[0, 1] == 0 and b[1, 1] == 1   # |k| = 1 -> 0.0156 < 0.02 ; sqrt2/64 > 0.02
    assert b[0, 25] == 1 and b[0, 26] == 0                   # 25/64 = 0.39 ; 26/64 = 0.406
    assert b[n - 25, 0] == 1 and b[32, 32] == 0              # negative frequency ; corner 0.707
    assert torch.equal(O.band_mask(n, 0.0, 0.0), torch.ones(n, n, dtype=F64))


# --------------------------------------------------------------- correlations

def _circ_corr_loops(f, g):
    n0, n1 = f.shape
    out = np.zeros((n0, n1))
    for sy in range(n0):
        for sx in range(n1):
            acc = 0.0
            for y in range(n0):
                for x in range(n1):
                    acc += f[y, x] * g[(y + sy) % n0, (x + sx) % n1]
            out[sy, sx] = acc
    return out


def test_cross_correlation_theorem():
    """iDFT(conj(F) G) equals the circular correlation sum of Eq. 3 (pure-Python loops)."""
    f, g = rnd(6, 6, seed=8), rnd(6, 6, seed=9)
    via_dft = O.idft2(O.dft2(f).conj() * O.dft2(g)).real.numpy()
    np.testing.assert_allclose(via_dft, _circ_corr_loops(f.numpy(), g.numpy()), atol=1e-11)


def test_linear_xy_correlation_padding():
    """ZeroPad to 2n + the theorem equals the linear correlation sum for every lag window entry."""
    n = 6
    f, g = rnd(n, n, seed=10), rnd(n, n, seed=11)
    fn, gn = f.numpy(), g.numpy()
    want = np.zeros((n, n))
    for iy, sy in enumerate(range(-n // 2, n // 2)):
        for ix, sx in enumerate(range(-n // 2, n // 2)):
            acc = 0.0
            for y in range(n):
                for x in range(n):
                    if 0 <= y + sy < n and 0 <= x + sx < n:
                        acc += fn[y, x] * gn[y + sy, x + sx]
            want[iy, ix] = acc
    np.testing.assert_allclose(O.xy_correlation_direct(f, g).numpy(), want, atol=1e-12)
    np.testing.assert_allclose(O.xy_correlation(f, g).numpy(), want, atol=1e-10)


def test_angle_correlation_sum_and_theorem():
    """Eq. 8 per radius: defining sum (pure Python) == oracle == per-radius DFT route averaged over r."""
    n_r, n_t = 3, 8
    pf, pg = rnd(n_r, n_t, seed=12), rnd(n_r, n_t, seed=13)
    a, b = pf.numpy(), pg.numpy()
    want = np.zeros(n_t)
    for k, l in enumerate(range(-n_t // 2, n_t // 2)):
        want[k] = sum(a[r, i] * b[r, (i + l) % n_t] for r in range(n_r) for i in range(n_t)) / n_r
    np.testing.assert_allclose(O.angle_correlation(pf, pg).numpy(), want, atol=1e-12)
    spec = (O.dft1(pf).conj() * O.dft1(pg)).sum(0) / n_r
    circ = O.idft1(spec[None, :])[0].real.numpy()
    np.testing.assert_allclose(circ[np.arange(-n_t // 2, n_t // 2) % n_t], want, atol=1e-12)


def test_correlation_symmetries():
    """c_theta(f, f) is even in the lag; c_xy(f, g)[s] = c_xy(g, f)[-s]."""
    n = 16
    f, g = rnd(n, n, seed=14).abs(), rnd(n, n, seed=15).abs()
    pf = O.cart2pol(O.dft2(f).abs(), n, n)
    c = O.angle_correlation(pf, pf).numpy()
    np.testing.assert_allclose(c[1:], c[1:][::-1], rtol=1e-12)
    cfg = O.xy_correlation(f, g).numpy()
    cgf = O.xy_correlation(g, f).numpy()
    np.testing.assert_allclose(cfg[1:, 1:], cgf[1:, 1:][::-1, ::-1], atol=1e-10)


# ----------------------------------------------------------------- closed forms

def test_delta_pair_gives_delta_surface():
    """Unit deltas at p and p + s: c_xy is 1 at lag s and 0 elsewhere."""
    n = 16
    f = torch.zeros(n, n, dtype=F64)
    g = torch.zeros(n, n, dtype=F64)
    f[5, 9] = 1.0
    g[5 + 3, 9 - 4] = 1.0
    c = O.xy_correlation(f, g)
    want = torch.zeros(n, n, dtype=F64)
    want[3 + n // 2, -4 + n // 2] = 1.0
    np.testing.assert_allclose(c.numpy(), want.numpy(), atol=1e-12)


@pytest.mark.parametrize("kind", ["delta", "zero"])
def test_flat_spectrum_gives_grid_mean(kind):
    """A centred delta has |F| = 1 everywhere and a zero scan has |F| = 0: c_theta is flat, so the
    soft-argmax returns the mean of the lag grid, -delta_theta/2 (even n)."""
    n = 16
    f = torch.zeros(n, n, dtype=F64)
    if kind == "delta":
        f[n // 2, n // 2] = 1.0
    p = O.Params(n=n, n_theta=n, delta_xy=0.5)
    out = O.search(f, f.clone(), p)
    ct = out["c_theta"].numpy()
    np.testing.assert_allclose(ct, ct[0], atol=1e-12)
    if kind == "delta":
        assert abs(ct[0] - n) < 1e-9     # (1/n_r) sum_b sum_a 1 * 1
    assert abs(float(out["theta"]) + math.pi / n / 2) < 1e-14
    if kind == "zero":
        # c_xy is flat too: t' is the grid mean (-d/2, -d/2), rotated by theta
        th = -math.pi / n / 2
        tp = np.array([-0.25, -0.25])
        want = np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]) @ tp
        np.testing.assert_allclose([float(out["tx"]), float(out["ty"])], want, atol=1e-12)


def _blob_scene(n, centres, amps, sigma=1.2):
    c = torch.arange(n, dtype=F64)
    img = torch.zeros(n, n, dtype=F64)
    for (r, q), a in zip(centres, amps):
        img += a * torch.exp(-((c[:, None] - r) ** 2 + (c[None, :] - q) ** 2) / (2 * sigma ** 2))
    return img


def test_integer_shift_is_recovered_exactly():
    """Compact scene, no window, pure integer translation: theta = 0 and t = s delta (Cauchy-Schwarz)."""
    n = 32
    f = _blob_scene(n, [(12, 14), (18, 11), (15, 20), (10, 9)], [1.0, 0.7, 0.5, 0.9])
    for s in [(3, -2), (-4, 5), (0, 1)]:
        g = torch.roll(f, shifts=s, dims=(0, 1))
        p = O.Params(n=n, n_theta=32, delta_xy=0.25, temp_theta=1e-6, temp_xy=1e-6, hann=False)
        out = O.search(f, g, p)
        assert int(torch.argmax(out["c_theta"])) == 16          # lag 0
        assert abs(float(out["theta"])) < 1e-12
        iy, ix = np.unravel_index(int(torch.argmax(out["c_xy"])), (n, n))
        assert (iy - n // 2, ix - n // 2) == s
        assert abs(float(out["tx"]) - 0.25 * s[1]) < 1e-9 and abs(float(out["ty"]) - 0.25 * s[0]) < 1e-9


def test_anisotropic_gaussian_heading():
    """A rotated elongated Gaussian has an analytically rotated spectrum: theta is recovered to a bin."""
    n, n_t = 64, 64
    c = torch.arange(n, dtype=F64) - n / 2
    X, Y = c[None, :], c[:, None]

    def ellipse(th):
        ct, st = math.cos(th), math.sin(th)
        u = ct * X + st * Y          # body axes of g at angle th
        v = -st * X + ct * Y
        return torch.exp(-(u ** 2) / (2 * 6.0 ** 2) - (v ** 2) / (2 * 1.5 ** 2))

    for th in [0.2, -0.35, 0.05]:
        f = ellipse(0.0)
        g = ellipse(th)        # g(R x) = f(x)  ->  Eq. 1 with theta* = th, t* = 0
        p = O.Params(n=n, n_theta=n_t, temp_theta=1e-3, temp_xy=1e-3, hann=False)
        out = O.search(f, g, p)
        assert abs(float(out["theta"]) - th) <= math.pi / n_t


def test_rotation_on_the_bin_grid():
    """Synthetic scene rotated by k bins, no translation, window on: error at most one bin."""
    spec = synth.SceneSpec(n=128, delta=0.5, n_reflectors=40, n_segments=10, speckle_sigma=0.1)
    n_t = 128
    for i, k in enumerate([3, -5, 7]):
        th = k * math.pi / n_t
        f, g, pose = synth.make_pair(spec, 99, "test", i, theta=th, t=(0.0, 0.0))
        p = O.Params(n=128, n_theta=n_t, delta_xy=0.5, band_lo=0.02, band_hi=0.4)
        out = O.search(f, g, p)
        assert abs(float(out["theta"]) - th) <= math.pi / n_t


def test_known_pose_pairs():
    """Eq. 1 end to end on generated pairs: heading within a bin, translation within pixels.

    The translation temperature is low here: raw correlation sums of these
    scenes differ by only a few units near the peak, so T = 1 averages over a
    broad neighbourhood and pulls t' toward the origin (that regime is the
    method's, but it would hide the frame conventions this test pins).
    """
    spec = synth.WORKLOADS["pair128"]
    th_err, t_err = [], []
    for i in range(8):
        f, g, pose = synth.make_pair(spec, 1, "val", i)
        p = O.Params(n=128, n_theta=128, delta_xy=0.5, band_lo=0.02, band_hi=0.4, temp_xy=0.05)
        est = O.search(f, g, p)["pose"].numpy()
        th_err.append(abs(est[0] - pose[0]))
        t_err.append(np.hypot(est[1] - pose[1], est[2] - pose[2]))
    assert max(th_err) <= math.pi / 128
    assert np.median(t_err) <= 0.5 and max(t_err) <= 1.5       # metres (1 px = 0.5 m)


def test_decoupled_search_agrees_with_joint_brute_force():
    """Eq. 2-3 brute force over (theta, t) vs the decoupled search: within one bin and one pixel."""
    n, n_t = 32, 64
    spec = synth.SceneSpec(n=n, delta=1.0, n_reflectors=12, n_segments=3, speckle_sigma=0.02,
                           theta_max_deg=12.0, t_max_m=3.0)
    for i in range(2):
        f, g, pose = synth.make_pair(spec, 98, "test", i)
        p = O.Params(n=n, n_theta=n_t, delta_xy=1.0, temp_theta=1e-3, temp_xy=1e-3)
        dec = O.search(f, g, p)
        thetas = [k * math.pi / n_t for k in range(-8, 9)]
        # the brute force of Eq. 2-3 correlates the scans themselves: a window on g would not
        # rotate with the scene and would pull the joint argmax toward theta = 0
        joint = O.joint_search(f, g, O.Params(n=n, n_theta=n_t, delta_xy=1.0, hann=False), thetas,
                               n_lag=12)
        assert abs(joint["theta"] - pose[0]) <= math.pi / n_t
        assert abs(joint["tx"] - pose[1]) <= 1.0 and abs(joint["ty"] - pose[2]) <= 1.0
        assert abs(float(dec["theta"]) - joint["theta"]) <= math.pi / n_t + 1e-12
        assert abs(float(dec["tx"]) - joint["tx"]) <= 1.0 + 1e-9
        assert abs(float(dec["ty"]) - joint["ty"]) <= 1.0 + 1e-9


def test_rotated_joint_matches_the_direct_joint_sums():
    """The comparator's scores J_k(s') (rotate g, FFT correlation) against the
    direct sums of Eq. 2, S_k(s) = sum_x fw(x) gw(R x + s): equal at s' = 0 for
    any heading, and entry for entry (s = R s') at the headings that map the
    lattice onto itself (-pi/2 and 0 among joint_headings(4))."""
    n = 12
    rng = np.random.Generator(np.random.PCG64(21))
    f = rng.uniform(0, 1, (n, n))
    g = rng.uniform(0, 1, (n, n))
    p = O.Params(n=n, n_theta=16, delta_xy=1.0, hann=True)
    th = O.joint_headings(4)
    j = O.joint_search_rotated(f, g, p, th)
    w = O.hann2d(n)
    fw, gw = w * torch.from_numpy(f), w * torch.from_numpy(g)
    S = O.joint_scores(fw, gw, [float(t) for t in th], n + 4)   # lags -n/2-2 .. n/2+1
    off = n // 2 + 2
    for k in range(4):
        assert abs(float(j["scores"][k, n // 2, n // 2] - S[k, off, off])) <= 1e-9 * float(S[k].abs().max())
    for k in (0, 2):                       # theta = -pi/2 and 0
        ct, st = round(math.cos(float(th[k]))), round(math.sin(float(th[k])))
        for iy in range(n):
            for ix in range(n):
                sy, sx = iy - n // 2, ix - n // 2
                rx, ry = ct * sx - st * sy, st * sx + ct * sy
                ref = S[k, ry + off, rx + off]
                assert abs(float(j["scores"][k, iy, ix] - ref)) <= 1e-9 * float(S[k].abs().max()), (k, iy, ix)


def test_rotated_joint_recovers_a_lattice_pose():
    """Sparse scene moved by an integer shift at a candidate heading of zero:
    the comparator's argmax is that heading and shift (Cauchy-Schwarz makes the
    true alignment the unique maximum)."""
    n = 16
    f = np.zeros((n, n))
    rng = np.random.Generator(np.random.PCG64(5))
    for _ in range(6):
        f[rng.integers(5, 11), rng.integers(5, 11)] += rng.uniform(0.5, 1.0)
    ty, tx = 2, -3
    g = np.roll(np.roll(f, ty, axis=0), tx, axis=1)       # g(y) = f(y - t): f(x) = g(x + t)
    p = O.Params(n=n, n_theta=16, delta_xy=0.5, hann=False)
    j = O.joint_search_rotated(f, g, p, O.joint_headings(8))
    assert j["theta"] == 0.0
    assert (j["tx"], j["ty"]) == (tx * 0.5, ty * 0.5)


# ------------------------------------------------------ full-circle heading

def test_full_circle_recovers_a_half_turn():
    """Compact scene turned by exactly pi about the centre pixel and shifted by
    whole pixels (a lattice permutation, so Eq. 1 holds exactly): the magnitude
    spectra coincide, stage 1 returns 0, and only the second stage-2 run, at
    -pi, finds the shift (Cauchy-Schwarz: its peak is the autocorrelation's)."""
    n = 32
    f = _blob_scene(n, [(12, 14), (18, 11), (15, 20), (10, 9)], [1.0, 0.7, 0.5, 0.9]).numpy()
    for ty, tx in [(2, -3), (-1, 4)]:
        # f(x) = g(R(pi) x + t)  <=>  g[i, j] = f[n + ty - i, n + tx - j]
        g = np.roll(np.flip(f, (0, 1)), (ty + 1, tx + 1), axis=(0, 1))
        p = O.Params(n=n, n_theta=32, delta_xy=0.25, temp_theta=1e-6, temp_xy=1e-6, hann=False)
        fc = O.search_full_circle(f, g, p)
        assert abs(float(fc["plain"][0])) < 1e-12
        assert fc["turned"] and float(fc["peaks"][1]) > float(fc["peaks"][0])
        th, px, py = [float(v) for v in fc["pose"]]
        assert abs(th + math.pi) < 1e-12
        assert abs(px - 0.25 * tx) < 1e-9 and abs(py - 0.25 * ty) < 1e-9
        # and the recovered pose maps g onto f on the lattice
        i, j = np.mgrid[0:n, 0:n]
        gi = np.rint(n / 2 + math.sin(th) * (j - n / 2) + math.cos(th) * (i - n / 2) + py / 0.25).astype(int)
        gj = np.rint(n / 2 + math.cos(th) * (j - n / 2) - math.sin(th) * (i - n / 2) + px / 0.25).astype(int)
        inside = (gi >= 0) & (gi < n) & (gj >= 0) & (gj < n)
        assert np.array_equal(g[gi[inside], gj[inside]], f[inside])
        assert np.abs(f[~inside]).max() < 1e-3 * f.max()     # the scene tails off before the edges


def test_full_circle_keeps_the_plain_search_when_it_wins():
    """Pure shift (heading 0): the first stage-2 run has the larger peak, and the
    pose is the plain search's, unchanged."""
    n = 32
    f = _blob_scene(n, [(12, 14), (18, 11), (15, 20), (10, 9)], [1.0, 0.7, 0.5, 0.9])
    g = torch.roll(f, shifts=(3, -2), dims=(0, 1))
    p = O.Params(n=n, n_theta=32, delta_xy=0.25, temp_theta=1e-6, temp_xy=1e-6, hann=False)
    fc = O.search_full_circle(f, g, p)
    assert not fc["turned"] and float(fc["peaks"][0]) > float(fc["peaks"][1])
    assert torch.equal(fc["pose"], O.search(f, g, p)["pose"])


def test_full_circle_on_generated_pairs_beyond_a_quarter_turn():
    """Generated pairs at headings past +-90 deg: the plain search returns the
    heading modulo pi, the full-circle search the heading itself (within a bin)
    and the translation (within pixels)."""
    spec = synth.WORKLOADS["pair128"]
    p = O.Params(n=128, n_theta=128, delta_xy=0.5, band_lo=0.02, band_hi=0.4, temp_xy=0.05)
    for i, th in enumerate([math.radians(150.0), math.radians(-125.0)]):
        f, g, pose = synth.make_pair(spec, 1, "val", i, theta=th)
        fc = O.search_full_circle(f, g, p)
        wrap = lambda a: (a + math.pi) % (2 * math.pi) - math.pi
        assert abs(wrap(float(fc["plain"][0]) - th + math.pi)) <= math.pi / 128
        assert fc["turned"]
        assert abs(wrap(float(fc["pose"][0]) - th)) <= math.pi / 128
        assert -math.pi <= float(fc["pose"][0]) < math.pi
        assert math.hypot(float(fc["pose"][1]) - pose[1], float(fc["pose"][2]) - pose[2]) <= 1.5


# -------------------------------------------------------------------- gradients

def test_gradient_matches_finite_differences():
    """Oracle autograd vs central differences on the FP64 forward, unsaturated temperatures."""
    n = 16
    rng = np.random.default_rng(21)
    f = torch.as_tensor(rng.random((n, n)), dtype=F64)
    g = torch.roll(f, shifts=(1, -1), dims=(0, 1)) + 0.05 * torch.as_tensor(rng.random((n, n)), dtype=F64)
    p = O.Params(n=n, n_theta=16, delta_xy=0.5, temp_theta=0.5, temp_xy=2.0, band_lo=0.05, band_hi=0.45)
    mf = torch.as_tensor(0.2 + 0.8 * rng.random((n, n)), dtype=F64)
    mg = torch.as_tensor(0.2 + 0.8 * rng.random((n, n)), dtype=F64)
    dpose = torch.tensor([0.7, -0.4, 0.9], dtype=F64)
    res = O.search_grad(f, g, dpose, p, mf, mg)

    def loss(ff, gg, a, b):
        return float((O.search(ff, gg, p, a, b)["pose"] * dpose).sum())

    h = 1e-6
    for (name, arr, idx) in [("d_f", f, (7, 8)), ("d_g", g, (9, 6)), ("d_m_f", mf, (8, 8)), ("d_m_g", mg, (6, 9))]:
        plus, minus = arr.clone(), arr.clone()
        plus[idx] += h
        minus[idx] -= h
        args_p = {"d_f": (plus, g, mf, mg), "d_g": (f, plus, mf, mg), "d_m_f": (f, g, plus, mg),
                  "d_m_g": (f, g, mf, plus)}[name]
        args_m = {"d_f": (minus, g, mf, mg), "d_g": (f, minus, mf, mg), "d_m_f": (f, g, minus, mg),
                  "d_m_g": (f, g, mf, minus)}[name]
        fd = (loss(*args_p) - loss(*args_m)) / (2 * h)
        ad = float(res[name][idx])
        assert abs(fd - ad) <= 1e-6 * max(1.0, abs(fd)), (name, fd, ad)


# ------------------------------------------------ alternative readings (options)

def _linear_corr_loops(fw, gp):
    """c[s] = sum_x fw[x] gp[x + s] over the lag window [-n/2, n/2)^2, zero outside (pure Python)."""
    n = fw.shape[0]
    out = np.zeros((n, n))
    for iy, sy in enumerate(range(-n // 2, n // 2)):
        for ix, sx in enumerate(range(-n // 2, n // 2)):
            acc = 0.0
            for y in range(n):
                for x in range(n):
                    if 0 <= y + sy < n and 0 <= x + sx < n:
                        acc += fw[y, x] * gp[y + sy, x + sx]
            out[iy, ix] = acc
    return out


def test_unwindowed_translation_stage():
    """With xy_unwindowed, stage 2 correlates the masked scans without the window
    (stage 1 keeps it): c_xy is the linear correlation of f m_f with g m_g rotated
    by the stage-1 heading, and the windowed reading gives a different surface."""
    n = 12
    r = np.random.default_rng(40)
    f, g = torch.tensor(r.random((n, n))), torch.tensor(r.random((n, n)))
    mf, mg = torch.tensor(r.random((n, n))), torch.tensor(r.random((n, n)))
    base = dict(n=n, n_theta=16, delta_xy=0.5, temp_theta=0.05, temp_xy=0.5, hann=True)
    un = O.search(f, g, O.Params(**base, xy_unwindowed=True), mf, mg)
    win = O.search(f, g, O.Params(**base), mf, mg)
    np.testing.assert_allclose(un["c_theta"].numpy(), win["c_theta"].numpy(), rtol=0, atol=1e-12)
    gp = O.rotate(g * mg, un["theta"]).numpy()
    want = _linear_corr_loops((f * mf).numpy(), gp)
    np.testing.assert_allclose(un["c_xy"].numpy(), want, rtol=0, atol=1e-10)
    assert float((un["c_xy"] - win["c_xy"]).abs().max()) > 1e-2 * float(un["c_xy"].abs().max())
    # the full-circle search's second run reads the same unwindowed scans
    fc = O.search_full_circle(f, g, O.Params(**base, xy_unwindowed=True), mf, mg)
    th = float(un["theta"])
    alt = th + math.pi if th < 0 else th - math.pi
    want2 = _linear_corr_loops((f * mf).numpy(), O.rotate(g * mg, torch.tensor(alt, dtype=F64)).numpy())
    np.testing.assert_allclose(fc["c_xy_turned"].numpy(), want2, rtol=0, atol=1e-10)


def test_marginal_angle_score_is_the_radius_mean_of_the_2d_correlation():
    """Algorithm 1's 'Mean over r' of the 2-D (radius, angle) circular correlation,
    computed here with numpy's FFT, is the marginal reading; with one radius the
    two readings coincide."""
    n_r, n_t = 5, 12
    pf, pg = rnd(n_r, n_t, seed=41), rnd(n_r, n_t, seed=42)
    c2 = np.fft.ifft2(np.conj(np.fft.fft2(pf.numpy())) * np.fft.fft2(pg.numpy())).real
    want = c2.mean(axis=0)[np.arange(-n_t // 2, n_t // 2) % n_t]
    np.testing.assert_allclose(O.angle_correlation_marginal(pf, pg).numpy(), want, rtol=0, atol=1e-12)
    np.testing.assert_allclose(O.angle_correlation_marginal(pf[:1], pg[:1]).numpy(),
                               O.angle_correlation(pf[:1], pg[:1]).numpy(), rtol=0, atol=1e-12)
    assert np.abs(O.angle_correlation(pf, pg).numpy() - want).max() > 1e-2


def test_marginal_reading_in_the_search():
    """The search's marginal option scores the polar spectra it resampled."""
    n = 16
    f, g = rnd(n, n, seed=43).abs(), rnd(n, n, seed=44).abs()
    out = O.search(f, g, O.Params(n=n, n_theta=16, angle_marginal=True))
    pf, pg = out["pf"].numpy(), out["pg"].numpy()
    n_t = pf.shape[1]
    c2 = np.fft.ifft2(np.conj(np.fft.fft2(pf)) * np.fft.fft2(pg)).real
    want = c2.mean(axis=0)[np.arange(-n_t // 2, n_t // 2) % n_t]
    np.testing.assert_allclose(out["c_theta"].numpy(), want, rtol=0, atol=1e-9)


@pytest.mark.parametrize("n_lags,temp", [(4, 1.0), (16, 0.5), (7, 2.0)])
def test_zscore_softmax_closed_form(n_lags, temp):
    """A one-hot score vector of n lags standardised by its mean and population
    standard deviation sqrt(n - 1) / n: the peak's logit exceeds every other by
    n / sqrt(n - 1), so p_peak = 1 / (1 + (n - 1) exp(-n / (sqrt(n - 1) T)))."""
    c = torch.zeros(n_lags, dtype=F64)
    c[2] = 3.7          # any positive height: standardisation removes it
    c = c - 11.0        # and any offset
    p = O.softmax_weights(c, temp, zscore=True)
    want = 1.0 / (1.0 + (n_lags - 1) * math.exp(-n_lags / (math.sqrt(n_lags - 1) * temp)))
    assert abs(float(p[2]) - want) < 1e-14
    np.testing.assert_allclose(p.sum().item(), 1.0, atol=1e-15)
    # without standardisation the raw height decides
    q = O.softmax_weights(c, temp, zscore=False)
    assert abs(float(q[2]) - 1.0 / (1.0 + (n_lags - 1) * math.exp(-3.7 / temp))) < 1e-14


def test_zscore_search_ignores_the_scale_of_the_scans():
    """Both score surfaces are linear in each scan, so standardised logits make the
    pose independent of a positive rescaling of f; raw logits do not."""
    n = 16
    f, g = rnd(n, n, seed=45).abs(), rnd(n, n, seed=46).abs()
    pz = O.Params(n=n, n_theta=16, delta_xy=0.5, temp_theta=0.5, temp_xy=0.5, zscore=True)
    pr = O.Params(n=n, n_theta=16, delta_xy=0.5, temp_theta=0.5, temp_xy=0.5)
    a, b = O.search(f, g, pz)["pose"], O.search(7.0 * f, g, pz)["pose"]
    np.testing.assert_allclose(a.numpy(), b.numpy(), rtol=0, atol=1e-12)
    a, b = O.search(f, g, pr)["pose"], O.search(7.0 * f, g, pr)["pose"]
    assert float((a - b).abs().max()) > 1e-3


# ------------------------------------------- odd sizes (127 / 255 / 511 px, 733 angle bins)

def test_centred_hann_is_the_periodic_hann_for_even_n_and_symmetric_for_odd_n():
    """The window written about the origin pixel c = floor(n/2) is the periodic Hann for
    even n; for odd n it peaks at c and is mirror symmetric about it."""
    for n in (16, 32, 128):
        np.testing.assert_allclose(O.hann_centred(n).numpy(), O.hann_periodic(n).numpy(), atol=1e-15)
    for n in (15, 127):
        h = O.hann_centred(n).numpy()
        c = n // 2
        assert h[c] == 1.0
        np.testing.assert_allclose(h[c + 1:], h[:c][::-1], atol=1e-15)
        # half a period from the peak the cosine is -cos(pi / n): the window is small but not zero
        assert abs(h[0] - 0.5 * (1.0 - math.cos(math.pi / n))) < 1e-15


def test_odd_size_spectra():
    """Parseval and shift invariance (Eq. 5-7) at odd sizes, against numpy's FFT."""
    for n in (15, 21):
        f = rnd(n, n, seed=40 + n)
        F = O.dft2(f)
        np.testing.assert_allclose(F.numpy(), np.fft.fft2(f.numpy()), atol=1e-10)
        assert abs(float((f ** 2).sum()) - float((F.abs() ** 2).sum()) / n ** 2) < 1e-10
        g = torch.roll(f, shifts=(4, -7), dims=(0, 1))
        np.testing.assert_allclose(O.dft2(g).abs().numpy(), F.abs().numpy(), atol=1e-10)


def test_odd_size_rotate_quarter_turn_about_the_origin_pixel():
    """For odd n the origin pixel c = (n - 1)/2 is the lattice centre, so a quarter turn maps
    every pixel onto a pixel: g'(y) = g(R y) reads column c - (i - c), row c + (j - c)."""
    n = 15
    c = n // 2
    g = rnd(n, n, seed=50)
    gq = O.rotate(g, torch.tensor(math.pi / 2, dtype=F64))
    for i in range(n):
        for j in range(n):
            # y = (j - c, i - c) -> R y = (-(i - c), j - c) -> column c - (i - c), row c + (j - c)
            assert abs(float(gq[i, j]) - float(g[c + (j - c), c - (i - c)])) < 1e-12


def test_odd_lag_grid_is_symmetric():
    """Odd n: lags -(n-1)/2 .. (n-1)/2, so a flat score surface averages to exactly zero
    (the even-n grid mean is -delta/2 instead)."""
    assert O.lag_indices(7).tolist() == [-3, -2, -1, 0, 1, 2, 3]
    n, n_t = 15, 9
    f = torch.zeros(n, n, dtype=F64)
    f[n // 2, n // 2] = 1.0                      # |F| = 1 everywhere: c_theta flat
    p = O.Params(n=n, n_theta=n_t, delta_xy=0.5)
    out = O.search(f, f.clone(), p)
    ct = out["c_theta"].numpy()
    np.testing.assert_allclose(ct, ct[0], atol=1e-12)
    assert abs(float(out["theta"])) < 1e-15
    z = O.search(torch.zeros(n, n, dtype=F64), torch.zeros(n, n, dtype=F64), p)
    assert abs(float(z["theta"])) < 1e-15 and abs(float(z["tx"])) < 1e-15 and abs(float(z["ty"])) < 1e-15


def test_odd_size_angle_correlation_defining_sum():
    """Eq. 8 at an odd number of bins (7): pure-Python circular sums over the symmetric lags."""
    n_r, n_t = 3, 7
    pf, pg = rnd(n_r, n_t, seed=51), rnd(n_r, n_t, seed=52)
    a, b = pf.numpy(), pg.numpy()
    want = [sum(a[r, i] * b[r, (i + l) % n_t] for r in range(n_r) for i in range(n_t)) / n_r
            for l in range(-3, 4)]
    np.testing.assert_allclose(O.angle_correlation(pf, pg).numpy(), want, atol=1e-12)


def test_odd_size_integer_shift_is_recovered_exactly():
    """Compact scene, no window, integer translation at n = 31: theta = 0 and t = s delta."""
    n = 31
    f = _blob_scene(n, [(12, 14), (18, 11), (15, 20), (10, 9)], [1.0, 0.7, 0.5, 0.9])
    for s in [(3, -2), (-4, 5)]:
        g = torch.roll(f, shifts=s, dims=(0, 1))
        p = O.Params(n=n, n_theta=33, delta_xy=0.25, temp_theta=1e-6, temp_xy=1e-6, hann=False)
        out = O.search(f, g, p)
        assert int(torch.argmax(out["c_theta"])) == 16          # lag 0 of 33
        assert abs(float(out["theta"])) < 1e-12
        iy, ix = np.unravel_index(int(torch.argmax(out["c_xy"])), (n, n))
        assert (iy - n // 2, ix - n // 2) == s
        assert abs(float(out["tx"]) - 0.25 * s[1]) < 1e-9 and abs(float(out["ty"]) - 0.25 * s[0]) < 1e-9


def test_odd_size_decoupled_search_agrees_with_joint_brute_force():
    """Eq. 2-3 brute force vs the decoupled search at n = 31: within a bin and a pixel; both
    land on the generator's pose (the origin pixel is shared by scenes, Rotate and lags)."""
    n, n_t = 31, 63
    spec = synth.SceneSpec(n=n, delta=1.0, n_reflectors=12, n_segments=3, speckle_sigma=0.02,
                           theta_max_deg=12.0, t_max_m=3.0)
    for i in range(2):
        f, g, pose = synth.make_pair(spec, 98, "test", i)
        p = O.Params(n=n, n_theta=n_t, delta_xy=1.0, temp_theta=1e-3, temp_xy=1e-3)
        dec = O.search(f, g, p)
        thetas = [k * math.pi / n_t for k in range(-8, 9)]
        joint = O.joint_search(f, g, O.Params(n=n, n_theta=n_t, delta_xy=1.0, hann=False), thetas,
                               n_lag=11)
        assert abs(joint["theta"] - pose[0]) <= math.pi / n_t
        assert abs(joint["tx"] - pose[1]) <= 1.0 and abs(joint["ty"] - pose[2]) <= 1.0
        assert abs(float(dec["theta"]) - joint["theta"]) <= math.pi / n_t + 1e-12
        assert abs(float(dec["tx"]) - joint["tx"]) <= 1.0 + 1e-9
        assert abs(float(dec["ty"]) - joint["ty"]) <= 1.0 + 1e-9


def test_generator_origin_is_the_origin_pixel():
    """The scene generator puts world (0, 0) at pixel (floor(n/2), floor(n/2)) for even and
    odd sides, the oracle's origin, and a point at (x, y) metres x / delta pixels to the right
    and y / delta rows down from it."""
    for n, d in ((127, 0.8), (128, 0.5), (511, 0.2)):
        np.testing.assert_allclose(synth._to_px(np.zeros(2), n, d), [n // 2, n // 2], atol=0)
        np.testing.assert_allclose(synth._to_px(np.array([2 * d, -3 * d]), n, d),
                                   [n // 2 + 2, n // 2 - 3], atol=1e-12)


def test_known_pose_pairs_at_the_papers_127_px():
    """Eq. 1 end to end at the paper's smallest size (127 px, 0.8 m/px, 733 bins, T_theta = 2):
    generated pairs come back within 1.5 degrees (median 0.5) and within a pixel.  At 127 px
    the magnitude spectra are coarse: the oracle's own heading error reaches about 1.2 degrees
    on these scenes at any temperature or bin count, while a sign or frame error would show
    up as about twice the heading (up to 20 degrees)."""
    spec = synth.WORKLOADS["paper127"]
    n_t = 733
    th_err, t_err = [], []
    for i in range(6):
        f, g, pose = synth.make_pair(spec, 5, "val", i)
        p = O.Params(n=127, n_theta=n_t, delta_xy=0.8, temp_theta=2.0, band_lo=0.02, band_hi=0.4,
                     temp_xy=0.05)
        est = O.search(f, g, p)["pose"].numpy()
        th_err.append(abs(est[0] - pose[0]))
        t_err.append(np.hypot(est[1] - pose[1], est[2] - pose[2]))
    assert max(th_err) <= math.radians(1.5) and np.median(th_err) <= math.radians(0.5)
    assert max(t_err) <= 0.8


def test_hard_argmax_reading_on_integer_shifts_and_ties():
    """The hard-argmax reading (Eq. 2-3 without the soft relaxation): integer shifts of a
    compact scene come back exactly (Cauchy-Schwarz: the correlation peaks at the shift),
    and among equal maxima the first in storage order wins."""
    n = 32
    f = _blob_scene(n, [(12, 14), (18, 11), (15, 20), (10, 9)], [1.0, 0.7, 0.5, 0.9])
    for s in [(3, -2), (-4, 5), (0, 1)]:
        g = torch.roll(f, shifts=s, dims=(0, 1))
        p = O.Params(n=n, n_theta=32, delta_xy=0.25, hann=False, hard_argmax=True)
        out = O.search(f, g, p)
        assert float(out["theta"]) == 0.0
        assert float(out["tx"]) == 0.25 * s[1] and float(out["ty"]) == 0.25 * s[0]
    w = O.argmax_weights(torch.tensor([[1.0, 3.0, 3.0], [0.0, 3.0, 2.0]], dtype=F64))
    assert w.tolist() == [[0.0, 1.0, 0.0], [0.0, 0.0, 0.0]]
