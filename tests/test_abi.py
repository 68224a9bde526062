"""Host-side checks of the C ABI: the library loads, exports every declared
symbol, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_2203_00459_amd import fmbym

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in sorted(os.listdir(os.path.join(ROOT, "include")))
           if h.endswith(".h")]


def declared_symbols():
    text = "".join(open(h).read() for h in HEADERS)
    return sorted(set(re.findall(r"FMBYM_API\s+[\w\s\*]+?\b(fmbym_\w+)\s*\(", text)))


def test_header_declares_the_binding_names():
    assert declared_symbols() == sorted(fmbym.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = fmbym.lib()
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = os.popen(f"nm -D --defined-only {fmbym.LIB_PATH}").read()
    exported = set(re.findall(r"\bT (\w+)", out))
    assert set(declared_symbols()) <= exported
    assert all(s.startswith("fmbym_") for s in exported if not s.startswith("_")), \
        sorted(s for s in exported if not s.startswith("fmbym_"))


def test_strerror():
    assert fmbym.strerror(0) == "success"
    assert "invalid" in fmbym.strerror(fmbym.FMBYM_EINVAL)
    assert "workspace" in fmbym.strerror(fmbym.FMBYM_EWORKSPACE)
    assert fmbym.strerror(12345) == "unknown error code"


GOOD = dict(n=128, n_theta=128, n_r=128, delta_xy=0.5, temp_theta=1.0, temp_xy=1.0, band_lo=0.02,
            band_hi=0.4, flags=fmbym.FMBYM_HANN)


@pytest.mark.parametrize("field,value,code", [
    ("n", 100, fmbym.FMBYM_EUNSUPPORTED),
    ("n", 0, fmbym.FMBYM_EINVAL),
    ("n_theta", 100, fmbym.FMBYM_EUNSUPPORTED),
    ("n_theta", 2048, fmbym.FMBYM_EUNSUPPORTED),
    ("n_r", 0, fmbym.FMBYM_EINVAL),
    ("n_r", 5000, fmbym.FMBYM_EUNSUPPORTED),
    ("delta_xy", 0.0, fmbym.FMBYM_EINVAL),
    ("temp_theta", -1.0, fmbym.FMBYM_EINVAL),
    ("temp_xy", float("nan"), fmbym.FMBYM_EINVAL),
    ("band_lo", 0.5, fmbym.FMBYM_EINVAL),
    ("flags", 1 << 9, fmbym.FMBYM_EUNSUPPORTED),
])
def test_plan_create_rejects_bad_parameters(field, value, code):
    kw = dict(GOOD)
    kw[field] = value
    p = fmbym.fmbym_params(*[kw[k] for k, _ in fmbym.fmbym_params._fields_])
    h = ctypes.c_void_p()
    rc = fmbym.lib().fmbym_plan_create(ctypes.byref(p), 1, ctypes.byref(h))
    assert rc == code and not h.value


def test_calls_without_a_plan_are_rejected():
    L = fmbym.lib()
    assert L.fmbym_search_workspace_size(None, 1, 0) == 0
    assert L.fmbym_search(None, 1, *([None] * 8), None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_backward(None, 1, *([None] * 13), None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_state_size(None, 1) == 0
    assert L.fmbym_joint_workspace_size(None, 1, 64) == 0
    t = fmbym.fmbym_tuning(8, 8, 8, 8, 1)
    assert L.fmbym_plan_get_tuning(None, ctypes.byref(t)) == fmbym.FMBYM_EINVAL
    assert L.fmbym_plan_set_tuning(None, ctypes.byref(t)) == fmbym.FMBYM_EINVAL
    assert L.fmbym_autotune_workspace_size(None, 1, 1) == 0
    assert L.fmbym_autotune(None, 1, 1, None, 0, None, ctypes.byref(t), None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_joint(None, 1, 64, *([None] * 6), None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_full_circle_workspace_size(None, 1) == 0
    assert L.fmbym_search_full_circle(None, 1, *([None] * 6), None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_train(None, 1, *([None] * 8), None, 0, None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_backward_state(None, 1, *([None] * 8), None, 0, *([None] * 5), None, 0,
                                         None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_search_vjp(None, 1, *([None] * 8), None, 0, *([None] * 5), None, 0,
                              None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_plan_destroy(None) == fmbym.FMBYM_EINVAL
    p = fmbym.fmbym_params(*[GOOD[k] for k, _ in fmbym.fmbym_params._fields_])
    assert L.fmbym_plan_create(ctypes.byref(p), 1, None) == fmbym.FMBYM_EINVAL
    h = ctypes.c_void_p()
    assert L.fmbym_plan_create(ctypes.byref(p), 0, ctypes.byref(h)) == fmbym.FMBYM_EINVAL


def test_ragged_calls_reject_bad_arguments():
    L = fmbym.lib()
    pairs = (fmbym.fmbym_pair * 1)()
    assert L.fmbym_ragged_workspace_size(None, 1, pairs, 1, None) == 0
    plans = (ctypes.c_void_p * 1)()
    assert L.fmbym_ragged_workspace_size(plans, 1, pairs, 1, None) == 0        # null plan
    assert L.fmbym_ragged_workspace_size(plans, 0, pairs, 1, None) == 0
    h = ctypes.c_void_p()
    assert L.fmbym_ragged_create(None, 1, pairs, 1, None, None, None, None, 0,
                                 ctypes.byref(h)) == fmbym.FMBYM_EINVAL
    assert L.fmbym_ragged_create(plans, 1, pairs, 1, None, None, None, None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_ragged_launch(None, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_ragged_destroy(None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_wall_clock_khz(None) == fmbym.FMBYM_EINVAL


def test_mask_calls_reject_bad_arguments():
    L = fmbym.lib()
    d = fmbym.fmbym_mask_desc(4, 8, 1e-5, 0.1, None, None, None)
    assert fmbym.mask_param_count(d) == 121_680 + 2 * 352 + 1
    assert fmbym.mask_bn_channels(d) == 352
    assert fmbym.mask_packed_bytes(d) > 2 * 121_608
    assert fmbym.mask_activation_bytes(d, 4, 64) == 0          # 64 >> 3 < 16 and n unsupported
    assert fmbym.mask_activation_bytes(d, 4, 128) > 0
    assert fmbym.mask_workspace_bytes(d, 0, 256) == 0
    bad = fmbym.fmbym_mask_desc(7, 8, 1e-5, 0.1, None, None, None)
    assert fmbym.mask_param_count(bad) == 0
    assert fmbym.mask_param_count(fmbym.fmbym_mask_desc(4, 8, 1e-5, 0.1, None, None, None, 3)) == 0
    six = fmbym.fmbym_mask_desc(6, 8, 1e-5, 0.1, None, None, None, 2)
    assert fmbym.mask_activation_bytes(six, 1, 256) == 0         # 256 >> 5 < 16
    assert fmbym.mask_activation_bytes(six, 1, 512) > 0
    assert L.fmbym_mask_fwd(ctypes.byref(bad), 1, 128, None, None, None, 0, 1, None) == fmbym.FMBYM_EUNSUPPORTED
    assert L.fmbym_mask_fwd(ctypes.byref(d), 1, 128, None, None, None, 0, 1, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_mask_bwd(None, 1, 128, None, None, 0, None, None, None, 0, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_mask_pack(ctypes.byref(d), None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_adam(None, None, None, None, 1, 1, 1e-3, 0.9, 0.999, 1e-8, None) == fmbym.FMBYM_EINVAL
    assert L.fmbym_pose_loss(1, None, None, 2, None, None, None) == fmbym.FMBYM_EINVAL


def test_mask_param_count_matches_the_oracle_layout():
    from oracle import mask_oracle as M
    for levels in (1, 2, 3, 4, 5, 6):
        for ch in (1, 2):
            d = fmbym.fmbym_mask_desc(levels, 8, 1e-5, 0.1, None, None, None, ch)
            assert fmbym.mask_param_count(d) == M.param_count(levels, 8, ch)
    # Table II's dual-input network: 1,965,024 convolution weights (about 1.97 M),
    # 1504 BatchNorm channels, two head biases
    d = fmbym.fmbym_mask_desc(6, 8, 1e-5, 0.1, None, None, None, 2)
    assert fmbym.mask_bn_channels(d) == 1504
    assert fmbym.mask_param_count(d) == 1_965_024 + 2 * 1504 + 2


def test_ragged_mix_counts_and_order():
    from paper_2203_00459_amd import synth, workloads
    cfg = workloads.RAGGED["ragged1024"]
    names = synth.ragged_mix(cfg["n_pairs"], cfg["mix"])
    assert len(names) == 1024
    assert (names.count("pair128"), names.count("batch256"), names.count("batch512")) == (513, 307, 204)
    assert names == synth.ragged_mix(cfg["n_pairs"], cfg["mix"])
    assert names[:8] != sorted(names[:8]) or names[8:16] != sorted(names[8:16])


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(fmbym, "_lib", None)
    monkeypatch.setattr(fmbym, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        fmbym.lib()
