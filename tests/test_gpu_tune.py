"""Column-tile widths, the batch split and the rows per line (the plan's
tuning) change speed, never results: the forward and the adjoint are bitwise
identical under every such choice for every supported n.  The radix plans of
the n-point column lines (radix 8 or 4) round differently: each is checked
against the FP64 oracle at the parity bar, and is bitwise invariant under the
other choices.  The autotuner returns choices from the supported set, sets them
on the plan, and its JSON cache gives them back without measuring again."""
import itertools

import numpy as np
import pytest
import torch

from paper_2203_00459_amd import fmbym, synth, tune, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
TUNINGS = [dict(cols1=c, cols2=c, cols_xy=c, cols_mag=c, split=1) for c in (4, 8)] + [
    dict(cols1=16, cols2=16, cols_xy=16, cols_mag=16, split=1, rows1=1, rows2=1),
    dict(cols1=16, cols2=4, cols_xy=8, cols_mag=4, split=2, rows1=1, rows2=2),
    dict(cols1=8, cols2=8, cols_xy=4, cols_mag=16, split=2, rows1=2, rows2=1)]


def _full(t):
    return dict(dict(rows1=2, rows2=2, radix1=8, radix_mag=8), **t)


@pytest.mark.parametrize("name", ["pair128", "batch256", "batch512"])
def test_every_width_gives_the_same_bits(name):
    B = 3   # an odd batch: the split's halves are 2 and 1 pairs
    print(f"case {name}", flush=True)
    s = fmbym.Search(max_batch=B, **workloads.search_kwargs(name))
    f, g, _ = synth.make_batch(name, B, split="val")
    f, g = torch.from_numpy(f).to(DEV), torch.from_numpy(g).to(DEV)
    rng = np.random.Generator(np.random.PCG64(2))
    mf, mg = (torch.from_numpy(rng.uniform(0.3, 1.0, f.shape).astype(np.float32)).to(DEV) for _ in range(2))
    d_pose = torch.from_numpy(rng.normal(size=(B, 3)).astype(np.float32)).to(DEV)
    ref = None
    for t in map(_full, TUNINGS):
        fmbym.plan_set_tuning(s.plan, t)
        assert fmbym.plan_get_tuning(s.plan) == t
        out = s.forward(f, g, mf, mg, keep=True)
        gr = s.backward(f, g, mf, mg, out, d_pose)
        torch.cuda.synchronize()
        res = {k: out[k].clone() for k in ("pose", "c_theta", "c_xy")}
        res.update({k: v.clone() for k, v in gr.items()})
        if ref is None:
            ref = res
            continue
        for k, v in res.items():
            assert torch.equal(v, ref[k]), (t, k)
    s.close()


@pytest.mark.parametrize("name", ["pair128", "batch256", "batch512"])
def test_radix_four_plans_match_the_oracle_and_are_width_invariant(name):
    """radix1 = radix_mag = 4: forward surfaces and pose, and the adjoint, at the
    parity bars against the oracle; bitwise the same under two other widths/splits."""
    from oracle import fmbym_oracle as O
    B = 2
    print(f"case {name} radix 4", flush=True)
    kw = dict(workloads.search_kwargs(name), temp_theta=5.0)
    s = fmbym.Search(max_batch=B, **kw)
    f, g, _ = synth.make_batch(name, B, split="val", start=2)
    F, G = torch.from_numpy(f).to(DEV), torch.from_numpy(g).to(DEV)
    d_pose = torch.tensor([[1.0, 0.0, 0.0]] * B, device=DEV)   # the rotation stage, through both tuned passes
    outs = []
    for t in (dict(cols1=4, cols_mag=4, split=1), dict(cols1=8, cols_mag=8, split=2, rows1=1)):
        fmbym.plan_set_tuning(s.plan, dict(t, radix1=4, radix_mag=4))
        out = s.forward(F, G, keep=True)
        gr = s.backward(F, G, None, None, out, d_pose)
        torch.cuda.synchronize()
        outs.append({k: v.clone() for k, v in list(out.items()) + list(gr.items()) if v is not None and k != "state"})
    for k, v in outs[0].items():
        assert torch.equal(v, outs[1][k]), k
    p = O.Params(**kw)
    o = outs[0]
    for b in range(B):
        ref = O.search(f[b], g[b], p)
        rc = ref["c_theta"] - ref["c_theta"].mean()
        e_t = float((o["c_theta"][b].double().cpu() - rc).abs().max() / rc.abs().max())
        e_x = float((o["c_xy"][b].double().cpu() - ref["c_xy"]).abs().max() / ref["c_xy"].abs().max())
        dp = np.abs(o["pose"][b].double().cpu().numpy() - ref["pose"].numpy())
        rg = O.search_grad(f[b], g[b], np.array([1.0, 0.0, 0.0]), p)
        e_g = max(float((o[k][b].double().cpu() - rg[k]).abs().max() / rg[k].abs().max()) for k in ("d_f", "d_g"))
        print(f"  pair {b}: c_theta {e_t:.2e} c_xy {e_x:.2e} dtheta {dp[0]:.1e} grad {e_g:.2e}", flush=True)
        assert e_t <= 1e-4 and e_x <= 1e-4 and dp[0] <= 1e-3 and max(dp[1:]) <= 1e-3 * kw["delta_xy"]
        assert e_g <= 1e-3
    s.close()


def test_set_tuning_rejects_unsupported_widths():
    s = fmbym.Search(max_batch=1, **workloads.search_kwargs("pair128"))
    with pytest.raises(fmbym.FmbymError):
        fmbym.plan_set_tuning(s.plan, dict(cols1=4, cols2=6, cols_xy=4, cols_mag=4, split=1))
    with pytest.raises(fmbym.FmbymError):
        fmbym.plan_set_tuning(s.plan, dict(cols1=4, cols2=4, cols_xy=4, cols_mag=4, split=3))
    with pytest.raises(fmbym.FmbymError):
        fmbym.plan_set_tuning(s.plan, dict(radix1=2))
    with pytest.raises(fmbym.FmbymError):
        fmbym.plan_set_tuning(s.plan, dict(rows1=3))
    s.close()
    big = fmbym.Search(max_batch=1, **workloads.search_kwargs("batch512"))
    with pytest.raises(fmbym.FmbymError):   # 16 columns of 512 points at radix 4: 2048 threads
        fmbym.plan_set_tuning(big.plan, dict(cols1=16, radix1=4))
    big.close()


def test_autotune_sets_supported_widths_and_caches(tmp_path):
    s = fmbym.Search(max_batch=8, **workloads.search_kwargs("batch256"))
    path = str(tmp_path / "tuning.json")
    r = tune.autotune(s, 8, with_backward=True, cache_path=path)
    print("autotune", r, flush=True)
    assert not r["from_cache"] and r["ms_per_step"] > 0
    assert all(r["tuning"][k] in (4, 8, 16) for k in ("cols1", "cols2", "cols_xy", "cols_mag"))
    assert r["tuning"]["split"] in (1, 2)
    assert r["tuning"]["rows1"] in (1, 2) and r["tuning"]["rows2"] in (1, 2)
    assert r["tuning"]["radix1"] in (4, 8) and r["tuning"]["radix_mag"] in (4, 8)
    assert fmbym.plan_get_tuning(s.plan) == r["tuning"]
    fmbym.plan_set_tuning(s.plan, dict(cols1=4, cols2=4, cols_xy=4, cols_mag=4, split=1, radix1=8, rows1=1))
    r2 = tune.autotune(s, 8, with_backward=True, cache_path=path)
    assert r2["from_cache"] and r2["tuning"] == r["tuning"]
    assert fmbym.plan_get_tuning(s.plan) == r["tuning"]
    s.close()
