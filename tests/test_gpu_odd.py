"""The forward search at the paper's odd sides (127, 255, 511 px) with its
ScanMatch defaults (733 heading bins, T_theta = 2) against the FP64 oracle,
which is pinned at odd sizes by its own tests.  Same bar as the even sizes:
surfaces max |dc| / max |c| <= 1e-4 per pair, pose within 1e-3 rad and
1e-3 px.  The heading scores come back centred (their mean over the lags in
saved[FMBYM_SAVED_THETA_MEAN])."""
import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SURF_TOL = 1e-4


def _inputs(name, B, masked=False, start=0):
    f, g, _ = synth.make_batch(name, B, split="val", start=start)
    mf = mg = None
    if masked:
        rng = np.random.default_rng(31)
        mf = rng.uniform(0.1, 1.0, f.shape).astype(np.float32)
        mg = rng.uniform(0.1, 1.0, f.shape).astype(np.float32)
    return f, g, mf, mg


def _dev(a):
    return None if a is None else torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _check(out, b, f, g, mf, mg, kw, label):
    ref = O.search(f, g, O.Params(**kw), mf, mg)
    ct = out["c_theta"][b].double().cpu()
    rc = ref["c_theta"] - ref["c_theta"].mean()
    cx = out["c_xy"][b].double().cpu()
    e_t = float((ct - rc).abs().max() / rc.abs().max())
    e_x = float((cx - ref["c_xy"]).abs().max() / ref["c_xy"].abs().max())
    mean = float(out["saved"][b, fmbym.FMBYM_SAVED_THETA_MEAN])
    e_m = abs(mean - float(ref["c_theta"].mean())) / float(ref["c_theta"].abs().max())
    dp = np.abs(out["pose"][b].double().cpu().numpy() - ref["pose"].numpy())
    print(f"{label} pair {b}: c_theta {e_t:.2e} c_xy {e_x:.2e} mean {e_m:.2e} "
          f"dtheta {dp[0]:.2e} rad dt {max(dp[1], dp[2]) / kw['delta_xy']:.2e} px", flush=True)
    assert e_t <= SURF_TOL and e_x <= SURF_TOL and e_m <= SURF_TOL
    assert dp[0] <= 1e-3 and max(dp[1], dp[2]) <= 1e-3 * kw["delta_xy"]


@pytest.mark.parametrize("name,B,masked,pairs", [
    ("paper127", 3, False, (0, 1, 2)), ("paper127", 2, True, (0, 1)),
    ("paper255", 2, False, (0, 1)), ("paper511", 4, False, (0, 3)),
])
def test_odd_forward_matches_oracle(name, B, masked, pairs):
    print(f"case {name} B={B} masked={masked}", flush=True)
    kw = workloads.search_kwargs(name)
    f, g, mf, mg = _inputs(name, B, masked)
    s = fmbym.Search(max_batch=B, **kw)
    out = s.forward(_dev(f), _dev(g), _dev(mf), _dev(mg))
    torch.cuda.synchronize()
    for b in pairs:
        _check(out, b, f[b], g[b], None if mf is None else mf[b], None if mg is None else mg[b], kw, name)
    s.close()


@pytest.mark.parametrize("n_theta,extra", [(16, {}), (128, {}), (1024, {}), (733, {"xy_unwindowed": True}),
                                           (733, {"hann": False})])
def test_odd_forward_other_bins_and_readings(n_theta, extra):
    """Every length of the heading line (16 -> 512 points, 128 -> 512, 1024 -> 2048,
    733 -> 1536), and stage 2 without the window, at 127 px."""
    print(f"case n_theta={n_theta} {extra}", flush=True)
    kw = dict(workloads.search_kwargs("paper127"), n_theta=n_theta, **extra)
    f, g, _, _ = _inputs("paper127", 2, start=4)
    s = fmbym.Search(max_batch=2, **kw)
    out = s.forward(_dev(f), _dev(g))
    torch.cuda.synchronize()
    for b in range(2):
        _check(out, b, f[b], g[b], None, None, kw, f"127/{n_theta}")
    s.close()


def test_odd_forward_is_deterministic_and_split_invariant():
    """Bitwise the same outputs on a repeat and with the batch split in two halves."""
    kw = workloads.search_kwargs("paper255")
    f, g, _, _ = _inputs("paper255", 5)
    F, G = _dev(f), _dev(g)
    s = fmbym.Search(max_batch=5, **kw)
    outs = []
    for split in (1, 1, 2):
        fmbym.plan_set_tuning(s.plan, dict(fmbym.plan_get_tuning(s.plan), split=split))
        o = s.forward(F, G)
        outs.append({k: v.clone() for k, v in o.items()})
    torch.cuda.synchronize()
    for o in outs[1:]:
        for k in ("pose", "c_theta", "c_xy", "saved"):
            assert torch.equal(o[k], outs[0][k]), k
    s.close()


def test_odd_plans_are_forward_only():
    """The adjoint, the training pair, the joint and full-circle searches, the
    autotuner and ragged lists report FMBYM_EUNSUPPORTED for odd sides; the
    checked-input flag is refused at plan creation."""
    kw = workloads.search_kwargs("paper127")
    s = fmbym.Search(max_batch=2, **kw)
    assert fmbym.search_workspace_size(s.plan, 2, True) == 0
    assert fmbym.search_state_size(s.plan, 2) == 0
    assert fmbym.joint_workspace_size(s.plan, 2, 8) == 0
    assert fmbym.full_circle_workspace_size(s.plan, 2) == 0
    f, g, _, _ = _inputs("paper127", 2)
    F, G = _dev(f), _dev(g)
    out = s.forward(F, G)
    with pytest.raises(fmbym.FmbymError) as e:
        s.backward(F, G, None, None, out, torch.ones(2, 3, device=DEV))
    assert e.value.code in (fmbym.FMBYM_EUNSUPPORTED, fmbym.FMBYM_EINVAL)
    with pytest.raises(fmbym.FmbymError):
        fmbym.plan_autotune(s.plan, 2, False, F.device)
    with pytest.raises(fmbym.FmbymError):
        fmbym.Ragged([s], [(F[0], G[0])])
    with pytest.raises(fmbym.FmbymError) as e:
        fmbym.Search(max_batch=1, check_finite=True, **kw)
    assert e.value.code == fmbym.FMBYM_EUNSUPPORTED
    s.close()
