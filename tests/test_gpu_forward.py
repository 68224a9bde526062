"""GPU parity of the forward search against the FP64 oracle.

Bar (written here, applied per pair):
  * surfaces: max |c_gpu - c_oracle| / max |c_oracle| <= 1e-4 for c_theta and c_xy;
  * pose: |theta_gpu - theta_oracle| <= 1e-3 rad, |t_gpu - t_oracle| <= 1e-3 px.
Small cases compare every pair; the full-size batches are run exactly as the
benchmark launches them and compared on sampled pairs.
"""
import math

import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

SURF_TOL = 1e-4
THETA_TOL = 1e-3
PX_TOL = 1e-3


def _compare(out, b, ref, delta):
    # c_theta comes back centred (its mean over lags in saved): compare both the
    # centred scores, which the softmax sees, and the recovered sums
    ct = out["c_theta"][b].double().cpu()
    mean = float(out["saved"][b, fmbym.FMBYM_SAVED_THETA_MEAN])
    ro = ref["c_theta"]
    rc = ro - ro.mean()
    e_c = float((ct - rc).abs().max() / rc.abs().max().clamp_min(1e-300))
    e_t = max(e_c, float((ct + mean - ro).abs().max() / ro.abs().max().clamp_min(1e-300)))
    cx = out["c_xy"][b].double().cpu()
    e_x = float((cx - ref["c_xy"]).abs().max() / ref["c_xy"].abs().max().clamp_min(1e-300))
    pose = out["pose"][b].double().cpu().numpy()
    rp = ref["pose"].numpy()
    d_th = abs(pose[0] - rp[0])
    d_t = max(abs(pose[1] - rp[1]), abs(pose[2] - rp[2])) / delta
    msg = (f"pair {b}: c_theta {e_t:.2e} (centred {e_c:.2e}) c_xy {e_x:.2e} dtheta {d_th:.2e} rad "
           f"dt {d_t:.2e} px")
    print(msg, flush=True)
    assert e_t <= SURF_TOL and e_x <= SURF_TOL, msg
    assert d_th <= THETA_TOL and d_t <= PX_TOL, msg


def _run(kw, f, g, mf=None, mg=None, max_batch=None):
    s = fmbym.Search(max_batch=max_batch or f.shape[0], **kw)
    dev = torch.device("cuda:0")
    t = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    out = s.forward(t(f), t(g), t(mf), t(mg))
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("case", ["pair128", "ragged", "masked", "n256_theta64_nohann", "unwindowed_xy",
                                  "theta16", "theta1024_r512"])
def test_forward_small_cases(case):
    print(f"case {case}", flush=True)
    kw = workloads.search_kwargs("pair128")
    B, mf, mg = 1, None, None
    name = "pair128"
    if case == "ragged":          # batch not a multiple of the 8-way XCD remap, n_r ragged vs radius blocks
        B = 3
        kw.update(n_r=100)
    elif case == "masked":
        B = 2
    elif case == "n256_theta64_nohann":
        name = "batch256"
        kw = workloads.search_kwargs("batch256")
        kw.update(n_theta=64, hann=False, temp_xy=0.5)
        B = 2
    elif case == "unwindowed_xy":
        kw.update(xy_unwindowed=True, temp_theta=3.0)
        B = 2
    elif case == "theta16":               # the smallest angle grid: one radius block holds 128 radii
        kw.update(n_theta=16, temp_theta=3.0)
        B = 2
    elif case == "theta1024_r512":        # the largest angle grid, radii denser than the scan's
        kw.update(n_theta=1024, n_r=512)
        B = 2
    f, g, _ = synth.make_batch(name, B, split="val", start=7)
    if case == "masked":
        rng = np.random.default_rng(5)
        mf = rng.uniform(0.05, 1.0, f.shape).astype(np.float32)
        mg = rng.uniform(0.05, 1.0, f.shape).astype(np.float32)
    out = _run(kw, f, g, mf, mg)
    p = O.Params(**kw)
    for b in range(B):
        ref = O.search(f[b], g[b], p, None if mf is None else mf[b], None if mg is None else mg[b])
        _compare(out, b, ref, kw["delta_xy"])


@pytest.mark.parametrize("name,samples", [("batch256", (0, 29, 63)), ("batch512", (0, 17, 31))])
def test_forward_full_batch_sampled(name, samples):
    print(f"workload {name}", flush=True)
    B = workloads.SEARCH[name]["batch"]
    kw = workloads.search_kwargs(name)
    f, g, _ = synth.make_batch(name, B, split="test")
    out = _run(kw, f, g)
    p = O.Params(**kw)
    for b in samples:
        _compare(out, b, O.search(f[b], g[b], p), kw["delta_xy"])


@pytest.mark.parametrize("kind", ["zero", "delta"])
def test_degenerate_inputs(kind):
    """Flat heading scores: the soft-argmax must return the lag-grid mean like the oracle.

    A centred delta has a flat magnitude spectrum only without the band-pass.
    """
    kw = workloads.search_kwargs("pair128")
    kw.update(band_lo=0.0, band_hi=0.0)
    n = kw["n"]
    f = np.zeros((2, n, n), np.float32)
    if kind == "delta":
        f[:, n // 2, n // 2] = 1.0
    out = _run(kw, f, f.copy())
    ref = O.search(f[0], f[0], O.Params(**kw))
    th = out["pose"][:, 0].double().cpu().numpy()
    assert np.all(np.abs(th - (-math.pi / kw["n_theta"] / 2)) < 1e-7)
    np.testing.assert_allclose(out["pose"][0].double().cpu().numpy(), ref["pose"].numpy(), atol=1e-6)


def test_bitwise_deterministic():
    kw = workloads.search_kwargs("batch256")
    f, g, _ = synth.make_batch("batch256", 8, split="val")
    a = _run(kw, f, g)
    b = _run(kw, f, g)
    for k in ("pose", "c_theta", "c_xy", "saved"):
        assert torch.equal(a[k], b[k]), k


def test_check_finite_counts_non_finite_inputs():
    """FMBYM_CHECK_FINITE: each pair's count of NaN / infinite values in f, g and
    the masks lands in saved[b][FMBYM_SAVED_STATUS] (counted here with numpy);
    a clean pair's outputs are bitwise those of a plan without the flag."""
    kw = workloads.search_kwargs("pair128")
    B = 3
    f, g, _ = synth.make_batch("pair128", B, split="val", start=11)
    rng = np.random.default_rng(8)
    mf = rng.uniform(0.2, 1.0, f.shape).astype(np.float32)
    mg = rng.uniform(0.2, 1.0, f.shape).astype(np.float32)
    f[1, 3, 5] = np.nan
    f[1, 100, 7] = np.inf
    g[1, 64, 64] = -np.inf
    mg[2, 0, 0] = np.nan
    mg[2, 127, 127] = np.nan
    mf[2, 50, 60] = np.inf
    want = [int((~np.isfinite(a[b])).sum() + (~np.isfinite(c[b])).sum() + (~np.isfinite(m1[b])).sum()
                + (~np.isfinite(m2[b])).sum()) for b in range(B) for a, c, m1, m2 in [(f, g, mf, mg)]]
    assert want == [0, 3, 3]
    checked = _run(dict(kw, check_finite=True), f, g, mf, mg)
    plain = _run(kw, f, g, mf, mg)
    got = [int(v) for v in checked["saved"][:, fmbym.FMBYM_SAVED_STATUS].cpu()]
    print("non-finite counts", got, flush=True)
    assert got == want
    for k in ("pose", "c_theta", "c_xy"):
        assert torch.equal(checked[k][0], plain[k][0]), k


@pytest.mark.parametrize("check", [False, True])
def test_every_saved_slot_is_written(check):
    """The forward defines all FMBYM_SAVED slots of every pair: the statistics,
    the status slot (0 without FMBYM_CHECK_FINITE, the count with it) and the
    reserved slots (0), whatever the buffer held before (NaN here)."""
    kw = dict(workloads.search_kwargs("pair128"), check_finite=check)
    B, n = 3, kw["n"]
    f, g, _ = synth.make_batch("pair128", B, split="val", start=5)
    dev = torch.device("cuda:0")
    s = fmbym.Search(max_batch=B, **kw)
    F, G = torch.from_numpy(f).to(dev), torch.from_numpy(g).to(dev)
    pose = torch.empty(B, 3, device=dev)
    saved = torch.full((B, fmbym.FMBYM_SAVED), float("nan"), device=dev)
    ws = s.workspace(B, False, dev)
    fmbym.search(s.plan, B, F.data_ptr(), G.data_ptr(), None, None, pose.data_ptr(), None, None,
                 saved.data_ptr(), ws.data_ptr(), ws.numel(), torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    sv = saved.cpu()
    print(f"check_finite={check} saved[0] = {sv[0].tolist()}", flush=True)
    assert bool(torch.isfinite(sv).all())
    assert bool((sv[:, fmbym.FMBYM_SAVED_STATUS:] == 0).all())
    ref = s.forward(F, G, surfaces=False)
    torch.cuda.synchronize()
    assert torch.equal(ref["pose"], pose)
    s.close()
