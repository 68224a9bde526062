"""The alternative readings of the scores, forward, against the FP64 oracle's
options: the marginal heading score (Alg. 1's "Mean over r" as the
correlation of radius-summed profiles), standardised logits (the temperature's
scale) and the hard argmax (Eq. 2-3 without the soft relaxation).  Bars as for
the default reading: surfaces max |dc| / max |c| <= 1e-4 per pair, poses within
1e-3 rad and 1e-3 px.  The hard argmax is an integer decision on FP32 scores:
it must equal the oracle's argmax wherever the oracle's top two scores differ by
more than the surfaces' bar, else be one of the near-tied maxima."""
import math

import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _run(name, B, masked=False, **flags):
    kw = dict(workloads.search_kwargs(name), **flags)
    f, g, _ = synth.make_batch(name, B, split="val", start=7)
    mf = mg = None
    if masked:
        rng = np.random.default_rng(41)
        mf = rng.uniform(0.2, 1.0, f.shape).astype(np.float32)
        mg = rng.uniform(0.2, 1.0, f.shape).astype(np.float32)
    s = fmbym.Search(max_batch=B, **kw)
    out = s.forward(_dev(f), _dev(g), _dev(mf), _dev(mg))
    torch.cuda.synchronize()
    return kw, f, g, mf, mg, out, s


def _surfaces(out, b, ref, label):
    ct = out["c_theta"][b].double().cpu()
    rc = ref["c_theta"] - ref["c_theta"].mean()
    cx = out["c_xy"][b].double().cpu()
    e_t = float((ct - rc).abs().max() / rc.abs().max())
    e_x = float((cx - ref["c_xy"]).abs().max() / ref["c_xy"].abs().max())
    print(f"{label} pair {b}: c_theta {e_t:.2e} c_xy {e_x:.2e}", flush=True)
    assert e_t <= 1e-4 and e_x <= 1e-4


@pytest.mark.parametrize("name,B,masked,flags", [
    ("pair128", 3, False, dict(angle_marginal=True)),
    ("batch256", 2, True, dict(angle_marginal=True)),
    ("pair128", 3, False, dict(zscore=True, temp_theta=0.5, temp_xy=0.5)),
    ("batch512", 2, False, dict(zscore=True, temp_theta=0.2, temp_xy=0.2)),
    ("batch256", 2, False, dict(angle_marginal=True, zscore=True, temp_theta=0.5, temp_xy=0.5)),
])
def test_soft_readings_match_the_oracle(name, B, masked, flags):
    print(f"case {name} B={B} masked={masked} {flags}", flush=True)
    kw, f, g, mf, mg, out, s = _run(name, B, masked, **flags)
    p = O.Params(**kw)
    for b in range(B):
        ref = O.search(f[b], g[b], p, None if mf is None else mf[b], None if mg is None else mg[b])
        _surfaces(out, b, ref, str(flags))
        dp = np.abs(out["pose"][b].double().cpu().numpy() - ref["pose"].numpy())
        print(f"  pose dtheta {dp[0]:.2e} rad dt {max(dp[1], dp[2]) / kw['delta_xy']:.2e} px", flush=True)
        assert dp[0] <= 1e-3 and max(dp[1], dp[2]) <= 1e-3 * kw["delta_xy"]
    s.close()


def _top_two_gap(c):
    v = torch.sort(c.reshape(-1), descending=True).values
    return float(v[0] - v[1]) / float(c.abs().max())


@pytest.mark.parametrize("name,B,flags", [("pair128", 4, {}), ("batch512", 2, {}),
                                          ("batch256", 2, dict(angle_marginal=True))])
def test_hard_argmax_matches_the_oracle(name, B, flags):
    print(f"case {name} B={B} hard {flags}", flush=True)
    kw, f, g, _, _, out, s = _run(name, B, hard_argmax=True, **flags)
    p = O.Params(**kw)
    for b in range(B):
        ref = O.search(f[b], g[b], p)
        _surfaces(out, b, ref, "hard")
        gpu = out["pose"][b].double().cpu().numpy()
        ref_pose = ref["pose"].numpy()
        gap_t, gap_x = _top_two_gap(ref["c_theta"]), _top_two_gap(ref["c_xy"])
        print(f"  pose {gpu} oracle {ref_pose} gaps {gap_t:.1e} {gap_x:.1e}", flush=True)
        if gap_t > 1e-4:
            assert gpu[0] == pytest.approx(ref_pose[0], abs=1e-7)
        else:   # one of the near-tied headings
            top = torch.nonzero(ref["c_theta"] >= ref["c_theta"].max() - 1e-4 * ref["c_theta"].abs().max())
            lags = (top.reshape(-1) - kw["n_theta"] // 2).double() * math.pi / kw["n_theta"]
            assert bool((lags - gpu[0]).abs().min() < 1e-7)
        if gap_t > 1e-4 and gap_x > 1e-4:
            assert np.abs(gpu[1:] - ref_pose[1:]).max() <= 1e-5 * kw["delta_xy"] + 1e-6
        # the heading is a lattice angle and the translation a rotated lattice lag
        k = gpu[0] / (math.pi / kw["n_theta"])
        assert abs(k - round(k)) < 1e-4
        c, sn = math.cos(gpu[0]), math.sin(gpu[0])
        tpx = (c * gpu[1] + sn * gpu[2]) / kw["delta_xy"]
        tpy = (-sn * gpu[1] + c * gpu[2]) / kw["delta_xy"]
        assert abs(tpx - round(tpx)) < 1e-3 and abs(tpy - round(tpy)) < 1e-3
    s.close()


def test_readings_are_forward_only():
    for flags in (dict(angle_marginal=True), dict(zscore=True), dict(hard_argmax=True)):
        s = fmbym.Search(max_batch=2, **dict(workloads.search_kwargs("pair128"), **flags))
        assert fmbym.search_workspace_size(s.plan, 2, True) == 0
        assert fmbym.search_state_size(s.plan, 2) == 0
        if not flags.get("angle_marginal"):
            assert fmbym.full_circle_workspace_size(s.plan, 2) > 0   # sized, but the call refuses
        s.close()
    with pytest.raises(fmbym.FmbymError) as e:
        fmbym.Search(max_batch=1, **dict(workloads.search_kwargs("paper127"), zscore=True))
    assert e.value.code == fmbym.FMBYM_EUNSUPPORTED
