"""The training forward (intermediates kept in a state buffer) and its adjoint
against the plain forward and the recomputing adjoint, on the same seeded
inputs: the outputs are the same kernels' results on the same values, so
they must agree bit for bit; the state is only read by the adjoint, so a
second adjoint call on it gives the same gradients again.  Both plain paths
are checked against the FP64 oracle in their own tests."""
import numpy as np
import pytest
import torch

from paper_2203_00459_amd import fmbym, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _inputs(name, B, masked):
    f, g, _ = synth.make_batch(name, B, split="val")
    f, g = torch.from_numpy(f).to(DEV), torch.from_numpy(g).to(DEV)
    if not masked:
        return f, g, None, None
    rng = np.random.Generator(np.random.PCG64(11))
    n = f.shape[-1]
    m = [torch.from_numpy(rng.uniform(0.2, 1.0, (B, n, n)).astype(np.float32)).to(DEV) for _ in range(2)]
    return f, g, m[0], m[1]


@pytest.mark.parametrize("name,B,masked", [("pair128", 2, False), ("pair128", 2, True),
                                           ("batch256", 3, True), ("batch512", 4, False)])
def test_state_path_equals_the_recomputing_path(name, B, masked):
    print(f"case {name} B={B} masked={masked}", flush=True)
    s = fmbym.Search(max_batch=B, **workloads.search_kwargs(name))
    f, g, mf, mg = _inputs(name, B, masked)
    ref = s.forward(f, g, mf, mg, surfaces=True)
    ref = {k: v.clone() for k, v in ref.items()}
    out = s.forward(f, g, mf, mg, keep=True)
    for k in ("pose", "c_theta", "c_xy", "saved"):
        assert torch.equal(out[k], ref[k]), k
    rng = np.random.Generator(np.random.PCG64(3))
    d_pose = torch.from_numpy(rng.normal(size=(B, 3)).astype(np.float32)).to(DEV)
    gr_ref = s.backward(f, g, mf, mg, ref, d_pose)
    gr_ref = {k: None if v is None else v.clone() for k, v in gr_ref.items()}
    for rep in range(2):
        gr = s.backward(f, g, mf, mg, out, d_pose)
        torch.cuda.synchronize()
        for k, v in gr_ref.items():
            if v is None:
                assert gr[k] is None
                continue
            d = float((gr[k] - v).abs().max()) / max(float(v.abs().max()), 1e-30)
            print(f"  rep {rep} {k}: max rel diff {d:.3e}", flush=True)
            assert torch.equal(gr[k], v), (rep, k, d)
    s.close()


def test_state_buffer_is_checked():
    s = fmbym.Search(max_batch=2, **workloads.search_kwargs("pair128"))
    f, g, _, _ = _inputs("pair128", 2, False)
    need = fmbym.search_state_size(s.plan, 2)
    assert need > 0
    st = torch.empty(need - 1, dtype=torch.uint8, device=DEV)
    o = {k: torch.empty(2, *sh, device=DEV) for k, sh in (("pose", (3,)), ("c_theta", (128,)),
                                                          ("c_xy", (128, 128)), ("saved", (fmbym.FMBYM_SAVED,)))}
    ws = s.workspace(2, False, f.device)
    with pytest.raises(fmbym.FmbymError):
        fmbym.search_train(s.plan, 2, f.data_ptr(), g.data_ptr(), None, None, o["pose"].data_ptr(),
                           o["c_theta"].data_ptr(), o["c_xy"].data_ptr(), o["saved"].data_ptr(), st.data_ptr(),
                           need - 1, ws.data_ptr(), ws.numel(), fmbym._stream())
    s.close()


@pytest.mark.parametrize("name,B,masked", [("pair128", 3, True), ("batch256", 3, False), ("batch512", 4, False)])
@pytest.mark.parametrize("split", [1, 2])
def test_vjp_equals_the_training_pair(name, B, masked, split):
    """fmbym_search_vjp (forward and adjoint per half, one fork and join) gives
    bit for bit what fmbym_search_train then fmbym_search_backward_state give."""
    print(f"case {name} B={B} masked={masked} split={split}", flush=True)
    s = fmbym.Search(max_batch=B, **workloads.search_kwargs(name))
    fmbym.plan_set_tuning(s.plan, dict(fmbym.plan_get_tuning(s.plan), split=split))
    f, g, mf, mg = _inputs(name, B, masked)
    d_pose = torch.from_numpy(np.random.Generator(np.random.PCG64(7)).normal(size=(B, 3))
                              .astype(np.float32)).to(DEV)
    fwd = s.forward(f, g, mf, mg, keep=True)
    grd = s.backward(f, g, mf, mg, fwd, d_pose)
    ref = {**{k: v.clone() for k, v in fwd.items()}, **{k: None if v is None else v.clone() for k, v in grd.items()}}
    out = s.vjp(f, g, mf, mg, d_pose)
    torch.cuda.synchronize()
    for k in ("pose", "c_theta", "c_xy", "saved", "d_f", "d_g", "d_m_f", "d_m_g"):   # state has padding
        if ref[k] is None:
            assert out[k] is None, k
            continue
        assert torch.equal(out[k], ref[k]), k
    s.close()


def test_vjp_buffers_are_checked():
    """fmbym_search_vjp rejects a state one byte short and a workspace one byte
    short of the adjoint's (which it needs), before enqueueing anything."""
    B = 2
    s = fmbym.Search(max_batch=B, **workloads.search_kwargs("batch256"))
    f, g, _, _ = _inputs("batch256", B, False)
    n, nt = s.n, s.n_theta
    o = {k: torch.empty(B, *sh, device=DEV) for k, sh in (("pose", (3,)), ("c_theta", (nt,)), ("c_xy", (n, n)),
                                                          ("saved", (fmbym.FMBYM_SAVED,)), ("d_pose", (3,)),
                                                          ("d_f", (n, n)), ("d_g", (n, n)))}
    need = fmbym.search_state_size(s.plan, B)
    st = torch.empty(need, dtype=torch.uint8, device=DEV)
    ws_full = fmbym.search_workspace_size(s.plan, B, True)
    ws = torch.empty(ws_full, dtype=torch.uint8, device=DEV)

    def call(state_bytes, ws_bytes):
        fmbym.search_vjp(s.plan, B, f.data_ptr(), g.data_ptr(), None, None, o["pose"].data_ptr(),
                         o["c_theta"].data_ptr(), o["c_xy"].data_ptr(), o["saved"].data_ptr(), st.data_ptr(),
                         state_bytes, o["d_pose"].data_ptr(), o["d_f"].data_ptr(), o["d_g"].data_ptr(), None,
                         None, ws.data_ptr(), ws_bytes, fmbym._stream())

    for state_bytes, ws_bytes in ((need - 1, ws_full), (need, ws_full - 1)):
        with pytest.raises(fmbym.FmbymError) as e:
            call(state_bytes, ws_bytes)
        assert e.value.code == fmbym.FMBYM_EWORKSPACE
    o["d_pose"].zero_()
    call(need, ws_full)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(o["d_f"]).all())
    s.close()
