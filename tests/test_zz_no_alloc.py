"""fmbym_search_noalloc (the forward with its workspace in the library's static
scratch array) against fmbym_search on the same inputs, through the C ABI: the
same kernels on the same values, so every output must agree bit for bit.  Two
calls in a row, the second with a smaller input, so the second reads an array
that still holds the first call's contents; then smaller and other plans on
the same array (256 px masked, 128 px, the 255 px odd side masked, standardised
logits)."""
import numpy as np
import pytest
import torch

from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _outputs(B, n, nt):
    return dict(pose=torch.full((B, 3), float("nan"), device=DEV),
                c_theta=torch.full((B, nt), float("nan"), device=DEV),
                c_xy=torch.full((B, n, n), float("nan"), device=DEV),
                saved=torch.full((B, fmbym.FMBYM_SAVED), float("nan"), device=DEV))


def _noalloc(s, f, g, mf, mg):
    B, n = f.shape[0], s.n
    o = _outputs(B, n, s.n_theta)
    fmbym.search_noalloc(s.plan, B, f.data_ptr(), g.data_ptr(), None if mf is None else mf.data_ptr(),
                         None if mg is None else mg.data_ptr(), o["pose"].data_ptr(), o["c_theta"].data_ptr(),
                         o["c_xy"].data_ptr(), o["saved"].data_ptr(), fmbym._stream())
    return o


def _inputs(name, B, masked, start=0):
    f, g, _ = synth.make_batch(name, B, split="val", start=start)
    f, g = torch.from_numpy(f).to(DEV), torch.from_numpy(g).to(DEV)
    if not masked:
        return f, g, None, None
    rng = np.random.default_rng(21 + start)
    n = f.shape[-1]
    return f, g, *[torch.from_numpy(rng.uniform(0.2, 1.0, (B, n, n)).astype(np.float32)).to(DEV)
                   for _ in range(2)]


def _compare(s, f, g, mf, mg, label):
    got = _noalloc(s, f, g, mf, mg)
    ref = s.forward(f, g, mf, mg, surfaces=True)
    torch.cuda.synchronize()
    for k in ("pose", "c_theta", "c_xy", "saved"):
        assert torch.equal(got[k], ref[k]), (label, k)
    print(f"{label}: bitwise equal to fmbym_search", flush=True)


@pytest.mark.parametrize("split", [1, 2])
def test_noalloc_equals_search_twice_smaller_second(split):
    s = fmbym.Search(max_batch=6, **workloads.search_kwargs("batch512"))
    fmbym.plan_set_tuning(s.plan, dict(fmbym.plan_get_tuning(s.plan), split=split))
    _compare(s, *_inputs("batch512", 6, False), f"512 B=6 split={split}")
    _compare(s, *_inputs("batch512", 3, False, start=6), f"512 B=3 split={split}")
    s.close()
    # a smaller scan size next, masked, on the same array
    s2 = fmbym.Search(max_batch=5, **workloads.search_kwargs("batch256"))
    fmbym.plan_set_tuning(s2.plan, dict(fmbym.plan_get_tuning(s2.plan), split=split))
    _compare(s2, *_inputs("batch256", 5, True), f"256 B=5 masked split={split}")
    s2.close()
    s3 = fmbym.Search(max_batch=1, **workloads.search_kwargs("pair128"))
    _compare(s3, *_inputs("pair128", 1, False), "128 B=1")
    s3.close()
    # the paper's odd side (its own kernels and workspace layout), masked, and a
    # plan with a reading flag whose scores pass through the workspace
    s4 = fmbym.Search(max_batch=2, **workloads.search_kwargs("paper255"))
    _compare(s4, *_inputs("paper255", 2, True), "255 B=2 masked")
    s4.close()
    s5 = fmbym.Search(max_batch=2, **dict(workloads.search_kwargs("batch256"), zscore=True))
    _compare(s5, *_inputs("batch256", 2, False, start=3), "256 B=2 zscore")
    s5.close()


def test_noalloc_rejects_a_batch_beyond_the_array():
    s = fmbym.Search(max_batch=64, **workloads.search_kwargs("batch512"))
    cap = fmbym.FMBYM_NOALLOC_SCRATCH_BYTES
    fits = [b for b in range(1, 65) if fmbym.search_workspace_size(s.plan, b, False) <= cap]
    big = max(fits) + 1
    assert 1 <= max(fits) < 64
    f, g, _, _ = _inputs("batch512", big, False)
    o = _outputs(big, 512, 512)
    with pytest.raises(fmbym.FmbymError) as e:
        fmbym.search_noalloc(s.plan, big, f.data_ptr(), g.data_ptr(), None, None, o["pose"].data_ptr(),
                             o["c_theta"].data_ptr(), o["c_xy"].data_ptr(), o["saved"].data_ptr(),
                             fmbym._stream())
    assert e.value.code == fmbym.FMBYM_EWORKSPACE
    torch.cuda.synchronize()
    assert torch.isnan(o["pose"]).all()     # nothing was enqueued
    # the largest batch that fits runs, and equals fmbym_search
    _compare(s, *_inputs("batch512", max(fits), False), f"512 B={max(fits)} (largest that fits)")
    s.close()
