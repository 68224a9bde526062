"""GPU parity of the hand-written adjoint against the FP64 oracle's autograd.

Conditioning.  Rotate resamples g bilinearly at R(theta) y, so d g'/d theta
is piecewise constant in theta, with a jump whenever one of the n^2 sample
positions crosses a lattice line: about every 1e-6 rad at 128 x 128.  The
heading gradient that flows through Rotate (dtheta_2) therefore changes by a
few percent between two evaluations whose theta differ by 1e-6 -- exactly the
difference between an FP32 and an FP64 forward.  Like an argmax near a tie,
that one scalar is compared for validity, not equality:
  * rotation stage alone (d_pose = e_theta) and translation stage alone
    (saturated heading softmax, so no gradient re-enters the rotation stage)
    are well conditioned and compared directly;
  * the full chain is compared after removing its component along G_rot, the
    gradient of a unit heading perturbation (the only direction a different
    dtheta_2 can move it); the removed coefficient must stay within the largest
    change of dtheta_2 that re-deciding the bilinear cells of sample positions
    near lattice lines can cause (a bound the oracle computes per pixel).

Bar: max |d_gpu - d_oracle| / max |d_oracle| <= GRAD_TOL, per pair and per
returned gradient.  The FP32 transforms carry ~1e-6 relative error, amplified
by 1/T through the softmax weights; 1e-3 leaves a wide margin while still
failing any dropped, mis-signed or mis-indexed term.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

GRAD_TOL = 1e-3
THETA_WINDOW = 2e-5       # |theta_gpu - theta_oracle| bound the full-chain check relies on (rad)


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _gpu_grad(kw, f, g, mf, mg, d_pose):
    s = fmbym.Search(max_batch=f.shape[0], **kw)
    F, G, MF, MG = _dev(f), _dev(g), _dev(mf), _dev(mg)
    out = s.forward(F, G, MF, MG)
    res = s.backward(F, G, MF, MG, out, _dev(d_pose))
    torch.cuda.synchronize()
    return out, res


def _err(a, ref):
    a = a.double().cpu()
    return float((a - ref).abs().max() / ref.abs().max().clamp_min(1e-300))


def _check_pair(res, b, ref, names, label=""):
    errs = {k: _err(res[k][b], ref[k]) for k in names}
    msg = f"{label} pair {b}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items())
    print(msg, flush=True)
    assert all(v <= GRAD_TOL for v in errs.values()), msg


def _case(case):
    name = "pair128"
    kw = workloads.search_kwargs("pair128")
    kw.update(temp_theta=5.0, temp_xy=1.0)
    if case == "n256_theta64":
        name = "batch256"
        kw = workloads.search_kwargs("batch256")
        kw.update(n_theta=64, temp_theta=20.0, temp_xy=2.0)
    if case == "unwindowed_xy":
        kw.update(xy_unwindowed=True)
    if case == "theta16":
        kw.update(n_theta=16, temp_theta=20.0)
    if case == "theta1024":
        kw.update(n_theta=1024, temp_theta=2.0)
    B = 2
    f, g, _ = synth.make_batch(name, B, split="val", start=3)
    mf = mg = None
    if case == "masked":
        rng = np.random.default_rng(13)      # masks whose heading scores have no near-tie
        mf = rng.uniform(0.1, 1.0, f.shape).astype(np.float32)
        mg = rng.uniform(0.1, 1.0, f.shape).astype(np.float32)
    return kw, f, g, mf, mg


CASES = ["plain", "masked", "unwindowed_xy", "n256_theta64", "theta16", "theta1024"]


@pytest.mark.parametrize("case", CASES)
def test_adjoint_rotation_stage(case):
    """d_pose = e_theta: only the heading soft-argmax, angular, polar and |F| adjoints act."""
    print(f"case {case}", flush=True)
    kw, f, g, mf, mg = _case(case)
    B = f.shape[0]
    d_pose = np.tile(np.array([1.0, 0.0, 0.0], np.float32), (B, 1))
    _, res = _gpu_grad(kw, f, g, mf, mg, d_pose)
    p = O.Params(**kw)
    names = ["d_f", "d_g"] + (["d_m_f", "d_m_g"] if mf is not None else [])
    for b in range(B):
        ref = O.search_grad(f[b], g[b], d_pose[b].astype(np.float64), p,
                            None if mf is None else mf[b], None if mg is None else mg[b])
        _check_pair(res, b, ref, names, "rotation")


def _saturating_temp(f, g, mf, mg, kw):
    """A heading temperature 40x below the oracle's smallest top-two score gap: the
    heading softmax is one-hot in both precisions and passes no gradient back."""
    p = O.Params(**kw)
    gaps = []
    for b in range(f.shape[0]):
        c = O.search(f[b], g[b], p, None if mf is None else mf[b], None if mg is None else mg[b])
        top = torch.sort(c["c_theta"], descending=True).values
        gaps.append(float(top[0] - top[1]))
    assert min(gaps) > 0.05, f"near-tied heading scores {gaps}: pick other pairs"
    return min(gaps) / 40.0


@pytest.mark.parametrize("case", CASES)
def test_adjoint_translation_stage(case):
    """Saturated heading softmax: translation adjoint, Rotate^T and the frame change only."""
    print(f"case {case}", flush=True)
    kw, f, g, mf, mg = _case(case)
    kw.update(temp_theta=_saturating_temp(f, g, mf, mg, kw))
    B = f.shape[0]
    d_pose = np.random.default_rng(1).standard_normal((B, 3)).astype(np.float32)
    _, res = _gpu_grad(kw, f, g, mf, mg, d_pose)
    p = O.Params(**kw)
    names = ["d_f", "d_g"] + (["d_m_f", "d_m_g"] if mf is not None else [])
    for b in range(B):
        ref = O.search_grad(f[b], g[b], d_pose[b].astype(np.float64), p,
                            None if mf is None else mf[b], None if mg is None else mg[b])
        _check_pair(res, b, ref, names, "translation")


def _dtheta2_flip_bound(f, g, d_pose, p, mf=None, mg=None):
    """Largest change of the Rotate-path heading gradient that re-deciding the
    bilinear cell of sample positions can cause, for every output pixel whose
    position lies within eps of a lattice line; eps covers a heading offset of
    THETA_WINDOW (times the pixel's speed d p / d theta) plus 1e-5 px of FP32
    position rounding.  Computed from the oracle alone."""
    ft = torch.as_tensor(f, dtype=torch.float64).clone().requires_grad_(True)
    gt = torch.as_tensor(g, dtype=torch.float64)
    o = O.search(ft, gt, p, mf, mg)
    loss = (o["pose"] * torch.as_tensor(d_pose, dtype=torch.float64)).sum()
    dgp = torch.autograd.grad(loss, o["gp"])[0].numpy()
    th = float(o["theta"])
    n = p.n
    g1 = g.astype(np.float64) * (1.0 if mg is None else mg.astype(np.float64))
    g2 = g1 if p.xy_unwindowed else (O.hann2d(n).numpy() * g1)
    pad = n                                              # rotated positions stay within n of the grid
    gp = np.pad(g2, pad)                                 # zero outside
    c, s = math.cos(th), math.sin(th)
    yy, yx = np.meshgrid(np.arange(n) - n // 2, np.arange(n) - n // 2, indexing="ij")
    px = c * yx - s * yy + n // 2
    py = s * yx + c * yy + n // 2
    vx = -s * yx - c * yy                                # d px / d theta
    vy = c * yx - s * yy
    eps = THETA_WINDOW * np.hypot(vx, vy) + 1e-5

    def term(y0, x0):
        wy, wx = py - y0, px - x0
        G = lambda dy, dx: gp[y0 + dy + pad, x0 + dx + pad]
        gx = (1 - wy) * (G(0, 1) - G(0, 0)) + wy * (G(1, 1) - G(1, 0))
        gy = (1 - wx) * (G(1, 0) - G(0, 0)) + wx * (G(1, 1) - G(0, 1))
        return gx * vx + gy * vy

    fy, fx = np.floor(py).astype(int), np.floor(px).astype(int)
    ry, rx = np.rint(py).astype(int), np.rint(px).astype(int)
    alt_y = np.where(np.abs(py - ry) < eps, np.where(fy == ry, ry - 1, ry), fy)
    alt_x = np.where(np.abs(px - rx) < eps, np.where(fx == rx, rx - 1, rx), fx)
    base = term(fy, fx)
    dev = np.maximum.reduce([np.abs(term(alt_y, fx) - base), np.abs(term(fy, alt_x) - base),
                             np.abs(term(alt_y, alt_x) - base)])
    return float((np.abs(dgp) * dev).sum()), th


def _full_chain_check(out, res, b, f, g, d_pose, p, label, mf=None, mg=None):
    ref = O.search_grad(f, g, d_pose, p, mf, mg)
    unit = O.search_grad(f, g, np.array([1.0, 0.0, 0.0]), p, mf, mg)   # gradient of a unit dtheta_total
    bound, th_o = _dtheta2_flip_bound(f, g, d_pose, p, mf, mg)
    d_th = abs(float(out["pose"][b, 0]) - th_o)
    assert d_th <= THETA_WINDOW, f"heading differs by {d_th:.2e} rad, beyond the window"
    names = ["d_f", "d_g"] + (["d_m_f", "d_m_g"] if mf is not None else [])
    r = torch.cat([(res[k][b].double().cpu() - ref[k]).reshape(-1) for k in names])
    G = torch.cat([unit[k].reshape(-1) for k in names])
    coef = float((r @ G) / (G @ G))
    resid = r - coef * G
    scale = float(torch.cat([ref[k].reshape(-1) for k in names]).abs().max())
    e = float(resid.abs().max()) / scale
    # the shift along G is visible only in proportion to |G|: allow the flip bound
    # plus whatever shift stays below the bar (G ~ 0 when the heading softmax is saturated)
    allow = 1.01 * bound + GRAD_TOL * scale / max(float(G.abs().max()), 1e-300)
    print(f"{label} pair {b}: residual {e:.2e}, dtheta_2 shift {coef:.3e} (allowed {allow:.3e}, "
          f"flip bound {bound:.3e}), dtheta {d_th:.1e}", flush=True)
    assert e <= GRAD_TOL
    assert abs(coef) <= allow


@pytest.mark.parametrize("case", ["plain", "unwindowed_xy", "n256_theta64"])
def test_adjoint_full_chain(case):
    print(f"case {case}", flush=True)
    kw, f, g, _, _ = _case(case)
    B = f.shape[0]
    d_pose = np.random.default_rng(1).standard_normal((B, 3)).astype(np.float32)
    out, res = _gpu_grad(kw, f, g, None, None, d_pose)
    p = O.Params(**kw)
    for b in range(B):
        _full_chain_check(out, res, b, f[b], g[b], d_pose[b].astype(np.float64), p, case)


def test_adjoint_full_batch512_sampled():
    """The benchmark's launch (32 pairs at 512 x 512, 512 bins), full chain, on sampled pairs."""
    name = "batch512"
    B = workloads.SEARCH[name]["batch"]
    kw = workloads.search_kwargs(name)
    f, g, _ = synth.make_batch(name, B, split="test")
    d_pose = np.ones((B, 3), np.float32)
    out, res = _gpu_grad(kw, f, g, None, None, d_pose)
    p = O.Params(**kw)
    for b in (0, 31):
        _full_chain_check(out, res, b, f[b], g[b], d_pose[b].astype(np.float64), p, "batch512")


@pytest.mark.parametrize("which,d_pose,temp_theta", [
    ("f", (1.0, 0.0, 0.0), 5.0), ("g", (1.0, 0.0, 0.0), 5.0),
    ("f", (0.0, 1.0, -1.0), 1e-4), ("g", (0.0, -0.5, 1.0), 1e-4),
])
def test_adjoint_directional_finite_differences(which, d_pose, temp_theta):
    """<grad, v> against central differences of the FP64 forward, h = 1e-3, on 8 x 8 patches."""
    kw = workloads.search_kwargs("pair128")
    kw.update(temp_theta=temp_theta, temp_xy=1.0)
    f, g, _ = synth.make_batch("pair128", 1, split="val", start=5)
    dp = np.array([d_pose], np.float32)
    _, res = _gpu_grad(kw, f, g, None, None, dp)
    p = O.Params(**kw)
    rng = np.random.default_rng(4)
    h = 1e-3
    base_f, base_g = f[0].astype(np.float64), g[0].astype(np.float64)
    grad = res["d_f" if which == "f" else "d_g"][0].double().cpu().numpy()
    for (r0, c0) in [(60, 60), (40, 70), (80, 30)]:
        v = np.zeros_like(base_f)
        v[r0:r0 + 8, c0:c0 + 8] = rng.standard_normal((8, 8))

        def loss(sign):
            ff = base_f + sign * h * v if which == "f" else base_f
            gg = base_g + sign * h * v if which == "g" else base_g
            return float((O.search(ff, gg, p)["pose"].numpy() * dp[0]).sum())

        fd = (loss(1) - loss(-1)) / (2 * h)
        ad = float((grad * v).sum())
        print(f"patch {which}{(r0, c0)} d_pose {d_pose}: fd {fd:.6e} adjoint {ad:.6e}", flush=True)
        assert abs(fd - ad) <= 1e-3 * max(abs(fd), 1e-4), (fd, ad)


def test_adjoint_bitwise_deterministic():
    kw = workloads.search_kwargs("batch256")
    f, g, _ = synth.make_batch("batch256", 4, split="val")
    d = np.ones((4, 3), np.float32)
    _, a = _gpu_grad(kw, f, g, None, None, d)
    _, b = _gpu_grad(kw, f, g, None, None, d)
    for k in ("d_f", "d_g"):
        assert torch.equal(a[k], b[k]), k


def test_autograd_function():
    """SearchFunction routes torch autograd through the library's adjoint."""
    kw = workloads.search_kwargs("pair128")
    kw.update(temp_theta=5.0)
    f, g, _ = synth.make_batch("pair128", 2, split="val")
    s = fmbym.Search(max_batch=2, **kw)
    F = _dev(f).requires_grad_(True)
    G = _dev(g).requires_grad_(True)
    pose = fmbym.SearchFunction.apply(s, F, G)
    (pose * torch.tensor([1.0, 2.0, -1.0], device="cuda:0")).sum().backward()
    d = np.tile(np.array([1.0, 2.0, -1.0], np.float32), (2, 1))
    _, res = _gpu_grad(kw, f, g, None, None, d)
    assert torch.equal(F.grad, res["d_f"]) and torch.equal(G.grad, res["d_g"])


# ------------------------------------------------------------ 512 x 512 (the benchmark's size)

C3_PAIRS = (0, 31)        # first and last pair of the benchmark's 32-pair batch
C3_TEMP_THETA = 20.0      # heading softmax unsaturated on both (largest weight 0.42 and 0.69)


def _c3_inputs():
    name = "batch512"
    kw = workloads.search_kwargs(name)
    kw.update(temp_theta=C3_TEMP_THETA)
    f, g, _ = synth.make_batch(name, workloads.SEARCH[name]["batch"], split="test")
    idx = list(C3_PAIRS)
    return kw, np.ascontiguousarray(f[idx]), np.ascontiguousarray(g[idx])


def _assert_unsaturated(f, g, p, mf=None, mg=None):
    """The heading softmax must spread its weight, or d theta / d input vanishes
    and the comparison could not see an error in the rotation-stage adjoint."""
    for b in range(f.shape[0]):
        o = O.search(f[b], g[b], p, None if mf is None else mf[b], None if mg is None else mg[b])
        pmax = float(O.softmax_weights(o["c_theta"], p.temp_theta, p.zscore).max())
        print(f"pair {b}: largest heading weight {pmax:.3f}", flush=True)
        assert 0.05 < pmax < 0.95, pmax


def _gpu_grad_state(kw, f, g, mf, mg, d_pose):
    """The training pair: forward keeping its intermediates, adjoint reading them."""
    s = fmbym.Search(max_batch=f.shape[0], **kw)
    F, G, MF, MG = _dev(f), _dev(g), _dev(mf), _dev(mg)
    out = s.forward(F, G, MF, MG, keep=True)
    res = s.backward(F, G, MF, MG, out, _dev(d_pose))
    torch.cuda.synchronize()
    return out, res


@pytest.mark.parametrize("path", ["recompute", "state"])
def test_adjoint_rotation_stage_512(path):
    """d_pose = e_theta at 512 x 512 with 512 bins and an unsaturated heading
    softmax: the polar, angular and |F| adjoints at the benchmark's size, on the
    recomputing adjoint and on the training pair's stored intermediates."""
    kw, f, g = _c3_inputs()
    p = O.Params(**kw)
    _assert_unsaturated(f, g, p)
    B = f.shape[0]
    d_pose = np.tile(np.array([1.0, 0.0, 0.0], np.float32), (B, 1))
    _, res = (_gpu_grad if path == "recompute" else _gpu_grad_state)(kw, f, g, None, None, d_pose)
    for b in range(B):
        ref = O.search_grad(f[b], g[b], d_pose[b].astype(np.float64), p)
        _check_pair(res, b, ref, ["d_f", "d_g"], f"rotation 512 {path}")


@pytest.mark.parametrize("path", ["recompute", "state"])
def test_adjoint_full_chain_512_unsaturated(path):
    """The whole chain at 512 x 512 with the heading softmax unsaturated, so the
    heading's gradient (both its paths) carries real weight."""
    kw, f, g = _c3_inputs()
    p = O.Params(**kw)
    B = f.shape[0]
    d_pose = np.random.default_rng(7).standard_normal((B, 3)).astype(np.float32)
    out, res = (_gpu_grad if path == "recompute" else _gpu_grad_state)(kw, f, g, None, None, d_pose)
    for b in range(B):
        _full_chain_check(out, res, b, f[b], g[b], d_pose[b].astype(np.float64), p, f"c3 {path}")


@pytest.mark.parametrize("which,d_pose,temp_theta", [
    ("f", (1.0, 0.0, 0.0), C3_TEMP_THETA), ("g", (1.0, 0.0, 0.0), C3_TEMP_THETA),
    ("f", (0.0, 1.0, -1.0), 1e-4), ("g", (0.0, -0.5, 1.0), 1e-4),
])
def test_adjoint_finite_differences_512(which, d_pose, temp_theta):
    """<grad, v> against central differences (h = 1e-3) of the FP64 forward on
    8 x 8 patches at 512 x 512: the heading (unsaturated softmax) and the
    translation (saturated heading, so theta is fixed).  The bar is normwise on
    the patch, 1e-3 |g_patch| |v| with g the oracle's gradient: a relative
    error e of the gradient moves <g, v> by at most e |g_patch| |v|, and a
    patch whose directional derivative happens to be small (one here is 5x
    below the others) must not tighten the bar on the gradient."""
    kw, f, g = _c3_inputs()
    kw.update(temp_theta=temp_theta)
    f, g = f[:1], g[:1]
    dp = np.array([d_pose], np.float32)
    _, res = _gpu_grad(kw, f, g, None, None, dp)
    p = O.Params(**kw)
    ref = O.search_grad(f[0], g[0], dp[0].astype(np.float64), p)["d_f" if which == "f" else "d_g"].numpy()
    rng = np.random.default_rng(12)
    h = 1e-3
    base_f, base_g = f[0].astype(np.float64), g[0].astype(np.float64)
    grad = res["d_f" if which == "f" else "d_g"][0].double().cpu().numpy()
    for (r0, c0) in [(252, 252), (180, 300), (310, 140)]:
        v = np.zeros_like(base_f)
        v[r0:r0 + 8, c0:c0 + 8] = rng.standard_normal((8, 8))

        def loss(sign):
            ff = base_f + sign * h * v if which == "f" else base_f
            gg = base_g + sign * h * v if which == "g" else base_g
            return float((O.search(ff, gg, p)["pose"].numpy() * dp[0]).sum())

        fd = (loss(1) - loss(-1)) / (2 * h)
        ad = float((grad * v).sum())
        scale = float(np.linalg.norm(ref[r0:r0 + 8, c0:c0 + 8]) * np.linalg.norm(v))
        print(f"512 patch {which}{(r0, c0)} d_pose {d_pose}: fd {fd:.6e} adjoint {ad:.6e} "
              f"|g_patch||v| {scale:.3e}", flush=True)
        assert abs(fd - ad) <= 1e-3 * scale, (fd, ad, scale)


def test_adjoint_full_chain_masked():
    """The whole chain with masks (Eq. 11): d_f, d_g, d_m_f and d_m_g at once."""
    kw, f, g, mf, mg = _case("masked")
    B = f.shape[0]
    d_pose = np.random.default_rng(5).standard_normal((B, 3)).astype(np.float32)
    out, res = _gpu_grad(kw, f, g, mf, mg, d_pose)
    p = O.Params(**kw)
    for b in range(B):
        _full_chain_check(out, res, b, f[b], g[b], d_pose[b].astype(np.float64), p, "masked",
                          mf[b], mg[b])
