"""Thin Python binding of libfmbym.so (C ABI in include/fmbym.h).

The functions with the C names only marshal arguments: every step of the
search runs in the library's HIP kernels.  ``Search`` adds the plumbing a
PyTorch caller wants (output and workspace tensors on the current stream), and
``SearchFunction`` exposes the hand-written adjoint to autograd.  There is no
fallback: if the library is missing this module raises on first use.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfmbym.so")

FMBYM_OK = 0
FMBYM_EINVAL = -1
FMBYM_EUNSUPPORTED = -2
FMBYM_EWORKSPACE = -3
FMBYM_EHIP = -4
FMBYM_HANN = 1
FMBYM_ANGLE_MARGINAL = 2
FMBYM_LOGIT_ZSCORE = 4
FMBYM_XY_UNWINDOWED = 8
FMBYM_HARD_ARGMAX = 16
FMBYM_CHECK_FINITE = 64
FMBYM_SAVED = 16
FMBYM_SAVED_THETA = 0
FMBYM_SAVED_COS = 1
FMBYM_SAVED_SIN = 2
FMBYM_SAVED_THETA_MAX = 3
FMBYM_SAVED_THETA_SUM = 4
FMBYM_SAVED_XY_MAX = 5
FMBYM_SAVED_XY_SUM = 6
FMBYM_SAVED_TPX = 7
FMBYM_SAVED_TPY = 8
FMBYM_SAVED_THETA_MEAN = 9
FMBYM_SAVED_THETA_ARG = 10
FMBYM_SAVED_THETA_NU = 11
FMBYM_SAVED_STATUS = 12

EXPORTS = (
    "fmbym_plan_create", "fmbym_plan_destroy", "fmbym_search_workspace_size", "fmbym_search",
    "fmbym_search_backward", "fmbym_strerror", "fmbym_last_hip_error", "fmbym_profile_enable",
    "fmbym_profile_read", "fmbym_ragged_workspace_size", "fmbym_ragged_create",
    "fmbym_ragged_launch", "fmbym_ragged_destroy", "fmbym_wall_clock_khz",
    "fmbym_mask_param_count", "fmbym_mask_packed_bytes", "fmbym_mask_bn_channels", "fmbym_mask_pack",
    "fmbym_mask_activation_bytes", "fmbym_mask_fwd", "fmbym_mask_workspace_bytes", "fmbym_mask_bwd",
    "fmbym_adam", "fmbym_pose_loss", "fmbym_search_state_size", "fmbym_search_train",
    "fmbym_search_backward_state", "fmbym_search_vjp", "fmbym_joint_workspace_size", "fmbym_search_joint",
    "fmbym_plan_get_tuning", "fmbym_plan_set_tuning", "fmbym_autotune_workspace_size", "fmbym_autotune",
    "fmbym_full_circle_workspace_size", "fmbym_search_full_circle", "fmbym_search_noalloc",
    "fmbym_search_ragged_workspace_size", "fmbym_search_ragged",
)
FMBYM_NOALLOC_SCRATCH_BYTES = 64 << 20
FMBYM_LOSS_L1 = 1
FMBYM_LOSS_L2 = 2


class fmbym_params(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("n_theta", ctypes.c_int32), ("n_r", ctypes.c_int32),
        ("delta_xy", ctypes.c_float), ("temp_theta", ctypes.c_float), ("temp_xy", ctypes.c_float),
        ("band_lo", ctypes.c_float), ("band_hi", ctypes.c_float), ("flags", ctypes.c_uint32),
    ]


FMBYM_PAIR_NET_MASK = 1


class fmbym_pair(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32), ("flags", ctypes.c_uint32), ("f", ctypes.c_void_p),
        ("g", ctypes.c_void_p), ("m_f", ctypes.c_void_p), ("m_g", ctypes.c_void_p),
    ]


class fmbym_tuning(ctypes.Structure):
    _fields_ = [("cols1", ctypes.c_int32), ("cols2", ctypes.c_int32), ("cols_xy", ctypes.c_int32),
                ("cols_mag", ctypes.c_int32), ("split", ctypes.c_int32), ("rows1", ctypes.c_int32),
                ("rows2", ctypes.c_int32), ("radix1", ctypes.c_int32), ("radix_mag", ctypes.c_int32)]


class fmbym_mask_desc(ctypes.Structure):
    _fields_ = [
        ("levels", ctypes.c_int32), ("base_channels", ctypes.c_int32), ("bn_eps", ctypes.c_float),
        ("bn_momentum", ctypes.c_float), ("params", ctypes.c_void_p), ("packed", ctypes.c_void_p),
        ("bn_running", ctypes.c_void_p), ("channels", ctypes.c_int32),
    ]


class FmbymError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = f"{where}: {strerror(code)} ({code})"
        if code == FMBYM_EHIP:
            msg += f", hipError {last_hip_error()}"
        super().__init__(msg)
        self.code = code


_lib = None


def lib() -> ctypes.CDLL:
    """Load the library (torch's HIP runtime is already in the process)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2203_00459_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, VP, SZ, I32 = ctypes.POINTER(fmbym_params), ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int32
        L.fmbym_plan_create.argtypes = [P, I32, ctypes.POINTER(VP)]
        L.fmbym_plan_create.restype = ctypes.c_int
        L.fmbym_plan_destroy.argtypes = [VP]
        L.fmbym_plan_destroy.restype = ctypes.c_int
        L.fmbym_search_workspace_size.argtypes = [VP, I32, ctypes.c_int]
        L.fmbym_search_workspace_size.restype = SZ
        L.fmbym_search.argtypes = [VP, I32] + [VP] * 8 + [VP, SZ, VP]
        L.fmbym_search.restype = ctypes.c_int
        L.fmbym_search_backward.argtypes = [VP, I32] + [VP] * 13 + [VP, SZ, VP]
        L.fmbym_search_backward.restype = ctypes.c_int
        TP = ctypes.POINTER(fmbym_tuning)
        L.fmbym_plan_get_tuning.argtypes = [VP, TP]
        L.fmbym_plan_get_tuning.restype = ctypes.c_int
        L.fmbym_plan_set_tuning.argtypes = [VP, TP]
        L.fmbym_plan_set_tuning.restype = ctypes.c_int
        L.fmbym_autotune_workspace_size.argtypes = [VP, I32, ctypes.c_int]
        L.fmbym_autotune_workspace_size.restype = SZ
        L.fmbym_autotune.argtypes = [VP, I32, ctypes.c_int, VP, SZ, VP, TP, ctypes.POINTER(ctypes.c_float)]
        L.fmbym_autotune.restype = ctypes.c_int
        L.fmbym_joint_workspace_size.argtypes = [VP, I32, I32]
        L.fmbym_joint_workspace_size.restype = SZ
        L.fmbym_search_joint.argtypes = [VP, I32, I32] + [VP] * 6 + [VP, SZ, VP]
        L.fmbym_search_joint.restype = ctypes.c_int
        L.fmbym_full_circle_workspace_size.argtypes = [VP, I32]
        L.fmbym_full_circle_workspace_size.restype = SZ
        L.fmbym_search_full_circle.argtypes = [VP, I32] + [VP] * 6 + [VP, SZ, VP]
        L.fmbym_search_full_circle.restype = ctypes.c_int
        L.fmbym_search_state_size.argtypes = [VP, I32]
        L.fmbym_search_state_size.restype = SZ
        L.fmbym_search_train.argtypes = [VP, I32] + [VP] * 8 + [VP, SZ, VP, SZ, VP]
        L.fmbym_search_train.restype = ctypes.c_int
        L.fmbym_search_backward_state.argtypes = [VP, I32] + [VP] * 8 + [VP, SZ] + [VP] * 5 + [VP, SZ, VP]
        L.fmbym_search_backward_state.restype = ctypes.c_int
        L.fmbym_search_vjp.argtypes = [VP, I32] + [VP] * 8 + [VP, SZ] + [VP] * 5 + [VP, SZ, VP]
        L.fmbym_search_vjp.restype = ctypes.c_int
        L.fmbym_search_noalloc.argtypes = [VP, I32] + [VP] * 8 + [VP]
        L.fmbym_search_noalloc.restype = ctypes.c_int
        L.fmbym_strerror.argtypes = [ctypes.c_int]
        L.fmbym_strerror.restype = ctypes.c_char_p
        L.fmbym_last_hip_error.argtypes = []
        L.fmbym_last_hip_error.restype = ctypes.c_int
        L.fmbym_profile_enable.argtypes = [I32]
        L.fmbym_profile_enable.restype = ctypes.c_int
        L.fmbym_profile_read.argtypes = [I32, ctypes.POINTER(ctypes.c_char_p),
                                         ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I32)]
        L.fmbym_profile_read.restype = ctypes.c_int
        PP = ctypes.POINTER(fmbym_pair)
        L.fmbym_ragged_workspace_size.argtypes = [ctypes.POINTER(VP), I32, PP, I32, VP]
        L.fmbym_ragged_workspace_size.restype = SZ
        L.fmbym_ragged_create.argtypes = [ctypes.POINTER(VP), I32, PP, I32, VP, VP, VP, VP, SZ,
                                          ctypes.POINTER(VP)]
        L.fmbym_ragged_create.restype = ctypes.c_int
        L.fmbym_search_ragged_workspace_size.argtypes = [ctypes.POINTER(VP), I32, PP, I32, VP]
        L.fmbym_search_ragged_workspace_size.restype = SZ
        L.fmbym_search_ragged.argtypes = [ctypes.POINTER(VP), I32, PP, I32, VP, VP, VP, VP, SZ, VP]
        L.fmbym_search_ragged.restype = ctypes.c_int
        L.fmbym_ragged_launch.argtypes = [VP, VP]
        L.fmbym_ragged_launch.restype = ctypes.c_int
        L.fmbym_ragged_destroy.argtypes = [VP]
        L.fmbym_ragged_destroy.restype = ctypes.c_int
        L.fmbym_wall_clock_khz.argtypes = [ctypes.POINTER(I32)]
        L.fmbym_wall_clock_khz.restype = ctypes.c_int
        MD = ctypes.POINTER(fmbym_mask_desc)
        for name in ("fmbym_mask_param_count", "fmbym_mask_packed_bytes", "fmbym_mask_bn_channels"):
            getattr(L, name).argtypes = [MD]
            getattr(L, name).restype = SZ
        L.fmbym_mask_pack.argtypes = [MD, VP]
        L.fmbym_mask_pack.restype = ctypes.c_int
        L.fmbym_mask_activation_bytes.argtypes = [MD, I32, I32]
        L.fmbym_mask_activation_bytes.restype = SZ
        L.fmbym_mask_workspace_bytes.argtypes = [MD, I32, I32]
        L.fmbym_mask_workspace_bytes.restype = SZ
        L.fmbym_mask_fwd.argtypes = [MD, I32, I32, VP, VP, VP, SZ, ctypes.c_int, VP]
        L.fmbym_mask_fwd.restype = ctypes.c_int
        L.fmbym_mask_bwd.argtypes = [MD, I32, I32, VP, VP, SZ, VP, VP, VP, SZ, VP]
        L.fmbym_mask_bwd.restype = ctypes.c_int
        L.fmbym_adam.argtypes = [VP, VP, VP, VP, ctypes.c_int64, I32, ctypes.c_float, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_float, VP]
        L.fmbym_adam.restype = ctypes.c_int
        L.fmbym_pose_loss.argtypes = [I32, VP, VP, I32, VP, VP, VP]
        L.fmbym_pose_loss.restype = ctypes.c_int
        _lib = L
    return _lib


# ------------------------------------------------------------ C-named calls

def strerror(code: int) -> str:
    return lib().fmbym_strerror(int(code)).decode()


def last_hip_error() -> int:
    return int(lib().fmbym_last_hip_error())


def plan_create(params: fmbym_params, max_batch: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = lib().fmbym_plan_create(ctypes.byref(params), int(max_batch), ctypes.byref(h))
    if rc:
        raise FmbymError(rc, "fmbym_plan_create")
    return h


def plan_destroy(plan) -> None:
    rc = lib().fmbym_plan_destroy(plan)
    if rc:
        raise FmbymError(rc, "fmbym_plan_destroy")


def search_workspace_size(plan, batch: int, with_backward: bool) -> int:
    return int(lib().fmbym_search_workspace_size(plan, int(batch), int(bool(with_backward))))


def search(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, workspace, workspace_bytes,
           stream) -> None:
    """fmbym_search with raw device addresses (ints or None)."""
    rc = lib().fmbym_search(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved, workspace,
                            int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search")


def search_noalloc(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, stream) -> None:
    """fmbym_search_noalloc (the forward on the library's static scratch array)."""
    rc = lib().fmbym_search_noalloc(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved, stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_noalloc")


def search_backward(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, d_pose, d_f, d_g,
                    d_m_f, d_m_g, workspace, workspace_bytes, stream) -> None:
    rc = lib().fmbym_search_backward(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved,
                                     d_pose, d_f, d_g, d_m_f, d_m_g, workspace, int(workspace_bytes),
                                     stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_backward")


TUNING_FIELDS = ("cols1", "cols2", "cols_xy", "cols_mag", "split", "rows1", "rows2", "radix1", "radix_mag")


def plan_get_tuning(plan) -> dict:
    t = fmbym_tuning()
    rc = lib().fmbym_plan_get_tuning(plan, ctypes.byref(t))
    if rc:
        raise FmbymError(rc, "fmbym_plan_get_tuning")
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}


def plan_set_tuning(plan, tuning: dict) -> None:
    """Replace the plan's launch choices; fields missing from `tuning` keep their value."""
    cur = plan_get_tuning(plan)
    t = fmbym_tuning(*[int(tuning.get(k, cur[k])) for k in TUNING_FIELDS])
    rc = lib().fmbym_plan_set_tuning(plan, ctypes.byref(t))
    if rc:
        raise FmbymError(rc, "fmbym_plan_set_tuning")


def plan_autotune(plan, batch: int, with_backward: bool, device) -> tuple[dict, float]:
    """Native autotune of the plan's column-tile widths; returns (widths, ms per step)."""
    need = int(lib().fmbym_autotune_workspace_size(plan, int(batch), int(with_backward)))
    if need == 0:
        raise FmbymError(FMBYM_EINVAL, "fmbym_autotune_workspace_size")
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    t = fmbym_tuning()
    ms = ctypes.c_float()
    rc = lib().fmbym_autotune(plan, int(batch), int(with_backward), ws.data_ptr(), need, _stream(),
                              ctypes.byref(t), ctypes.byref(ms))
    if rc:
        raise FmbymError(rc, "fmbym_autotune")
    return {k: int(getattr(t, k)) for k in TUNING_FIELDS}, float(ms.value)


def joint_workspace_size(plan, batch, n_angles) -> int:
    return int(lib().fmbym_joint_workspace_size(plan, int(batch), int(n_angles)))


def search_joint(plan, batch, n_angles, f, g, m_f, m_g, pose, peak, workspace, workspace_bytes, stream) -> None:
    """fmbym_search_joint with raw device addresses (ints or None)."""
    rc = lib().fmbym_search_joint(plan, int(batch), int(n_angles), f, g, m_f, m_g, pose, peak, workspace,
                                  int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_joint")


def full_circle_workspace_size(plan, batch) -> int:
    return int(lib().fmbym_full_circle_workspace_size(plan, int(batch)))


def search_full_circle(plan, batch, f, g, m_f, m_g, pose, peaks, workspace, workspace_bytes, stream) -> None:
    """fmbym_search_full_circle with raw device addresses (ints or None)."""
    rc = lib().fmbym_search_full_circle(plan, int(batch), f, g, m_f, m_g, pose, peaks, workspace,
                                        int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_full_circle")


def search_state_size(plan, batch) -> int:
    return int(lib().fmbym_search_state_size(plan, int(batch)))


def search_train(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, state, state_bytes, workspace,
                 workspace_bytes, stream) -> None:
    """fmbym_search_train with raw device addresses (ints or None)."""
    rc = lib().fmbym_search_train(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved, state,
                                  int(state_bytes), workspace, int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_train")


def search_backward_state(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, state, state_bytes,
                          d_pose, d_f, d_g, d_m_f, d_m_g, workspace, workspace_bytes, stream) -> None:
    rc = lib().fmbym_search_backward_state(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved,
                                           state, int(state_bytes), d_pose, d_f, d_g, d_m_f, d_m_g,
                                           workspace, int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_backward_state")


def search_vjp(plan, batch, f, g, m_f, m_g, pose, c_theta, c_xy, saved, state, state_bytes, d_pose, d_f, d_g,
               d_m_f, d_m_g, workspace, workspace_bytes, stream) -> None:
    """fmbym_search_vjp with raw device addresses (ints or None)."""
    rc = lib().fmbym_search_vjp(plan, int(batch), f, g, m_f, m_g, pose, c_theta, c_xy, saved, state,
                                int(state_bytes), d_pose, d_f, d_g, d_m_f, d_m_g, workspace,
                                int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_vjp")


def profile_enable(capacity: int) -> None:
    rc = lib().fmbym_profile_enable(int(capacity))
    if rc:
        raise FmbymError(rc, "fmbym_profile_enable")


def profile_read() -> dict:
    """{kernel name: (total ms, launches)} for kernels launched since profile_enable."""
    K = 64
    names = (ctypes.c_char_p * K)()
    ms = (ctypes.c_double * K)()
    cnt = (ctypes.c_int32 * K)()
    rc = lib().fmbym_profile_read(K, names, ms, cnt)
    if rc < 0:
        raise FmbymError(rc, "fmbym_profile_read")
    return {names[k].decode(): (ms[k], cnt[k]) for k in range(rc) if cnt[k] > 0}


def _plan_array(plans):
    arr = (ctypes.c_void_p * len(plans))()
    for k, p in enumerate(plans):
        arr[k] = p.value if isinstance(p, ctypes.c_void_p) else p
    return arr


def ragged_workspace_size(plans, pairs, net=None) -> int:
    """plans: plan handles; pairs: a ctypes array of fmbym_pair; net: fmbym_mask_desc or None."""
    return int(lib().fmbym_ragged_workspace_size(_plan_array(plans), len(plans), pairs, len(pairs),
                                                 None if net is None else ctypes.addressof(net)))


def ragged_create(plans, pairs, pose, stamps, workspace, workspace_bytes, net=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    rc = lib().fmbym_ragged_create(_plan_array(plans), len(plans), pairs, len(pairs),
                                   None if net is None else ctypes.addressof(net), pose, stamps,
                                   workspace, int(workspace_bytes), ctypes.byref(h))
    if rc:
        raise FmbymError(rc, "fmbym_ragged_create")
    return h


def search_ragged_workspace_size(plans, pairs, net=None) -> int:
    return int(lib().fmbym_search_ragged_workspace_size(_plan_array(plans), len(plans), pairs, len(pairs),
                                                        None if net is None else ctypes.addressof(net)))


def search_ragged(plans, pairs, pose, stamps, workspace, workspace_bytes, stream, net=None) -> None:
    """fmbym_search_ragged: the work list searched in one call (no launch object)."""
    rc = lib().fmbym_search_ragged(_plan_array(plans), len(plans), pairs, len(pairs),
                                   None if net is None else ctypes.addressof(net), pose, stamps, workspace,
                                   int(workspace_bytes), stream)
    if rc:
        raise FmbymError(rc, "fmbym_search_ragged")


def ragged_launch(ragged, stream) -> None:
    rc = lib().fmbym_ragged_launch(ragged, stream)
    if rc:
        raise FmbymError(rc, "fmbym_ragged_launch")


def ragged_destroy(ragged) -> None:
    rc = lib().fmbym_ragged_destroy(ragged)
    if rc:
        raise FmbymError(rc, "fmbym_ragged_destroy")


def wall_clock_khz() -> int:
    v = ctypes.c_int32()
    rc = lib().fmbym_wall_clock_khz(ctypes.byref(v))
    if rc:
        raise FmbymError(rc, "fmbym_wall_clock_khz")
    return int(v.value)


# ------------------------------------------------------------------ plumbing

def _ptr(t: torch.Tensor | None, shape=None, name=""):
    if t is None:
        return None
    if t.device.type != "cuda" or t.dtype != torch.float32 or not t.is_contiguous():
        raise ValueError(f"{name}: expected a contiguous float32 device tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Search:
    """A plan plus torch-allocated outputs and workspace for one parameter set."""

    def __init__(self, n: int, n_theta: int, n_r: int | None = None, delta_xy: float = 1.0,
                 temp_theta: float = 1.0, temp_xy: float = 1.0, band_lo: float = 0.0,
                 band_hi: float = 0.0, hann: bool = True, xy_unwindowed: bool = False,
                 check_finite: bool = False, max_batch: int = 64, angle_marginal: bool = False,
                 zscore: bool = False, hard_argmax: bool = False):
        flags = ((FMBYM_HANN if hann else 0) | (FMBYM_XY_UNWINDOWED if xy_unwindowed else 0)
                 | (FMBYM_CHECK_FINITE if check_finite else 0) | (FMBYM_ANGLE_MARGINAL if angle_marginal else 0)
                 | (FMBYM_LOGIT_ZSCORE if zscore else 0) | (FMBYM_HARD_ARGMAX if hard_argmax else 0))
        self.params = fmbym_params(n, n_theta, n if n_r is None else n_r, delta_xy, temp_theta,
                                   temp_xy, band_lo, band_hi, flags)
        self.n, self.n_theta, self.max_batch = n, n_theta, max_batch
        self.plan = plan_create(self.params, max_batch)
        self._ws = None
        self._jws = None

    def close(self):
        if self.plan is not None:
            plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, batch: int, with_backward: bool, device) -> torch.Tensor:
        need = search_workspace_size(self.plan, batch, with_backward)
        if need == 0:
            raise FmbymError(FMBYM_EINVAL, "fmbym_search_workspace_size")
        if self._ws is None or self._ws.numel() < need or self._ws.device != device:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device)
        return self._ws

    def forward(self, f, g, m_f=None, m_g=None, surfaces: bool = True, keep: bool = False) -> dict:
        """keep=True: the training forward, which also returns ``state`` (the
        intermediates the adjoint then reads instead of recomputing)."""
        B, n = f.shape[0], self.n
        dev = f.device
        if keep:
            return self._forward_keep(f, g, m_f, m_g)
        out = dict(pose=torch.empty(B, 3, device=dev),
                   c_theta=torch.empty(B, self.n_theta, device=dev) if surfaces else None,
                   c_xy=torch.empty(B, n, n, device=dev) if surfaces else None,
                   saved=torch.empty(B, FMBYM_SAVED, device=dev))
        ws = self.workspace(B, False, dev)
        search(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
               _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"), _ptr(out["pose"]),
               _ptr(out["c_theta"]), _ptr(out["c_xy"]), _ptr(out["saved"]), ws.data_ptr(),
               ws.numel(), _stream())
        return out

    def joint(self, f, g, n_angles: int, m_f=None, m_g=None) -> dict:
        """The brute-force joint comparator: pose [B, 3] and peak [B, n_angles]."""
        B, n = f.shape[0], self.n
        dev = f.device
        need = joint_workspace_size(self.plan, B, n_angles)
        if need == 0:
            raise FmbymError(FMBYM_EINVAL, "fmbym_joint_workspace_size")
        if self._jws is None or self._jws.numel() < need or self._jws.device != dev:
            self._jws = torch.empty(need, dtype=torch.uint8, device=dev)
        out = dict(pose=torch.empty(B, 3, device=dev), peak=torch.empty(B, n_angles, device=dev))
        search_joint(self.plan, B, n_angles, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                     _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"), _ptr(out["pose"]),
                     _ptr(out["peak"]), self._jws.data_ptr(), need, _stream())
        return out

    def full_circle(self, f, g, m_f=None, m_g=None) -> dict:
        """Heading over the whole circle: pose [B, 3] and peaks [B, 2] (max c_xy at
        theta and at theta + pi)."""
        B, n = f.shape[0], self.n
        dev = f.device
        need = full_circle_workspace_size(self.plan, B)
        if need == 0:
            raise FmbymError(FMBYM_EINVAL, "fmbym_full_circle_workspace_size")
        if self._jws is None or self._jws.numel() < need or self._jws.device != dev:
            self._jws = torch.empty(need, dtype=torch.uint8, device=dev)
        out = dict(pose=torch.empty(B, 3, device=dev), peaks=torch.empty(B, 2, device=dev))
        search_full_circle(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                           _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"), _ptr(out["pose"]),
                           _ptr(out["peaks"]), self._jws.data_ptr(), need, _stream())
        return out

    def _forward_keep(self, f, g, m_f, m_g) -> dict:
        B, n = f.shape[0], self.n
        dev = f.device
        need = search_state_size(self.plan, B)
        out = dict(pose=torch.empty(B, 3, device=dev), c_theta=torch.empty(B, self.n_theta, device=dev),
                   c_xy=torch.empty(B, n, n, device=dev), saved=torch.empty(B, FMBYM_SAVED, device=dev),
                   state=torch.empty(need, dtype=torch.uint8, device=dev))
        ws = self.workspace(B, False, dev)
        search_train(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                     _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"), _ptr(out["pose"]),
                     _ptr(out["c_theta"]), _ptr(out["c_xy"]), _ptr(out["saved"]), out["state"].data_ptr(),
                     need, ws.data_ptr(), ws.numel(), _stream())
        return out

    def vjp(self, f, g, m_f, m_g, d_pose) -> dict:
        """Training forward and adjoint in one call for a given d_pose: the
        outputs of forward(keep=True) and of backward on them, in one dict."""
        B, n = f.shape[0], self.n
        dev = f.device
        need = search_state_size(self.plan, B)
        out = dict(pose=torch.empty(B, 3, device=dev), c_theta=torch.empty(B, self.n_theta, device=dev),
                   c_xy=torch.empty(B, n, n, device=dev), saved=torch.empty(B, FMBYM_SAVED, device=dev),
                   state=torch.empty(need, dtype=torch.uint8, device=dev),
                   d_f=torch.empty(B, n, n, device=dev), d_g=torch.empty(B, n, n, device=dev),
                   d_m_f=None if m_f is None else torch.empty(B, n, n, device=dev),
                   d_m_g=None if m_g is None else torch.empty(B, n, n, device=dev))
        ws = self.workspace(B, True, dev)
        search_vjp(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                   _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"), _ptr(out["pose"]),
                   _ptr(out["c_theta"]), _ptr(out["c_xy"]), _ptr(out["saved"]), out["state"].data_ptr(), need,
                   _ptr(d_pose.contiguous(), (B, 3), "d_pose"), _ptr(out["d_f"]), _ptr(out["d_g"]),
                   _ptr(out["d_m_f"]), _ptr(out["d_m_g"]), ws.data_ptr(), ws.numel(), _stream())
        return out

    def backward(self, f, g, m_f, m_g, fwd: dict, d_pose) -> dict:
        """The adjoint; reads fwd["state"] when the forward kept one."""
        B, n = f.shape[0], self.n
        dev = f.device
        res = dict(d_f=torch.empty(B, n, n, device=dev), d_g=torch.empty(B, n, n, device=dev),
                   d_m_f=None if m_f is None else torch.empty(B, n, n, device=dev),
                   d_m_g=None if m_g is None else torch.empty(B, n, n, device=dev))
        ws = self.workspace(B, True, dev)
        st = fwd.get("state")
        if st is not None:
            search_backward_state(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                                  _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"),
                                  _ptr(fwd["pose"]), _ptr(fwd["c_theta"]), _ptr(fwd["c_xy"]),
                                  _ptr(fwd["saved"]), st.data_ptr(), st.numel(),
                                  _ptr(d_pose.contiguous(), (B, 3), "d_pose"), _ptr(res["d_f"]),
                                  _ptr(res["d_g"]), _ptr(res["d_m_f"]), _ptr(res["d_m_g"]), ws.data_ptr(),
                                  ws.numel(), _stream())
            return res
        search_backward(self.plan, B, _ptr(f, (B, n, n), "f"), _ptr(g, (B, n, n), "g"),
                        _ptr(m_f, (B, n, n), "m_f"), _ptr(m_g, (B, n, n), "m_g"),
                        _ptr(fwd["pose"]), _ptr(fwd["c_theta"]), _ptr(fwd["c_xy"]),
                        _ptr(fwd["saved"]), _ptr(d_pose.contiguous(), (B, 3), "d_pose"),
                        _ptr(res["d_f"]), _ptr(res["d_g"]), _ptr(res["d_m_f"]), _ptr(res["d_m_g"]),
                        ws.data_ptr(), ws.numel(), _stream())
        return res


class SearchFunction(torch.autograd.Function):
    """pose = search(f, g[, m_f, m_g]) with the library's hand-written adjoint."""

    @staticmethod
    def forward(ctx, searcher: Search, f, g, m_f=None, m_g=None):
        out = searcher.forward(f, g, m_f, m_g, surfaces=True)
        ctx.searcher = searcher
        ctx.fwd = out
        ctx.save_for_backward(f, g, m_f, m_g)
        return out["pose"]

    @staticmethod
    def backward(ctx, d_pose):
        f, g, m_f, m_g = ctx.saved_tensors
        r = ctx.searcher.backward(f, g, m_f, m_g, ctx.fwd, d_pose)
        return None, r["d_f"], r["d_g"], r["d_m_f"], r["d_m_g"]


def pair_array(pairs, net=None):
    """A ctypes fmbym_pair array of (f, g), (f, g, m_f, m_g) or (f, g, "net")
    device tensors, and their device."""
    arr = (fmbym_pair * len(pairs))()
    dev = None
    for i, q in enumerate(pairs):
        f, g = q[0], q[1]
        n = f.shape[-1]
        if len(q) == 3 and isinstance(q[2], str):
            if q[2] != "net" or net is None:
                raise ValueError("a (f, g, 'net') pair needs the net argument")
            arr[i] = fmbym_pair(n, FMBYM_PAIR_NET_MASK, _ptr(f, (n, n), "f"), _ptr(g, (n, n), "g"), None, None)
        else:
            m_f, m_g = (q[2], q[3]) if len(q) > 2 else (None, None)
            arr[i] = fmbym_pair(n, 0, _ptr(f, (n, n), "f"), _ptr(g, (n, n), "g"),
                                _ptr(m_f, (n, n), "m_f"), _ptr(m_g, (n, n), "m_g"))
        dev = f.device
    return arr, dev


def ragged_search(searches, pairs, net: "MaskNet | None" = None, stamps: bool = False):
    """The one-call ragged search (fmbym_search_ragged): poses [P, 3] of a mixed
    list of pairs, as ``Ragged`` would give them, without a launch object.
    With stamps, returns (poses, stamps [P + 1])."""
    arr, dev = pair_array(pairs, net)
    plans = [s.plan for s in searches]
    desc = None if net is None else net.desc
    need = search_ragged_workspace_size(plans, arr, desc)
    if need == 0:
        raise FmbymError(FMBYM_EINVAL, "fmbym_search_ragged_workspace_size")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    pose = torch.empty(len(pairs), 3, device=dev)
    st = torch.zeros(len(pairs) + 1, dtype=torch.int64, device=dev) if stamps else None
    search_ragged(plans, arr, pose.data_ptr(), None if st is None else st.data_ptr(), ws.data_ptr(), need,
                  _stream(), desc)
    return (pose, st) if stamps else pose


class Ragged:
    """A ragged work list (pairs of mixed sizes) as one replayable launch.

    ``searches`` are Search objects with distinct n; ``pairs`` is a list of
    (f, g), (f, g, m_f, m_g) or (f, g, "net") device tensors, each [n, n] for
    one of those n; "net" takes the masks from ``net`` (a MaskNet, run in
    inference mode inside the launch).  The tensors must stay alive and in
    place: every launch reads them anew.  ``pose`` [P, 3] and ``stamps`` [P + 1]
    (int64 wall-clock ticks, the last one the launch start) are refreshed by
    every launch.
    """

    def __init__(self, searches, pairs, stamps: bool = True, net: "MaskNet | None" = None):
        self.searches = list(searches)
        self.net = net
        self._keep = list(pairs)
        arr, dev = pair_array(pairs, net)
        plans = [s.plan for s in self.searches]
        desc = None if net is None else net.desc
        need = ragged_workspace_size(plans, arr, desc)
        if need == 0:
            raise FmbymError(FMBYM_EINVAL, "fmbym_ragged_workspace_size")
        self.workspace = torch.empty(need, dtype=torch.uint8, device=dev)
        self.pose = torch.zeros(len(pairs), 3, device=dev)
        self.stamps = torch.zeros(len(pairs) + 1, dtype=torch.int64, device=dev) if stamps else None
        self.handle = ragged_create(plans, arr, self.pose.data_ptr(),
                                    None if self.stamps is None else self.stamps.data_ptr(),
                                    self.workspace.data_ptr(), need, desc)

    def launch(self) -> torch.Tensor:
        ragged_launch(self.handle, _stream())
        return self.pose

    def latencies_us(self) -> torch.Tensor:
        """Per-pair time from the launch start to its pose write, in microseconds."""
        s = self.stamps.cpu()
        return (s[:-1] - s[-1]).double() * 1e3 / wall_clock_khz()

    def close(self):
        if getattr(self, "handle", None) is not None:
            ragged_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------- mask network

def _check(rc: int, where: str) -> None:
    if rc:
        raise FmbymError(rc, where)


def mask_param_count(desc: fmbym_mask_desc) -> int:
    return int(lib().fmbym_mask_param_count(ctypes.byref(desc)))


def mask_packed_bytes(desc: fmbym_mask_desc) -> int:
    return int(lib().fmbym_mask_packed_bytes(ctypes.byref(desc)))


def mask_bn_channels(desc: fmbym_mask_desc) -> int:
    return int(lib().fmbym_mask_bn_channels(ctypes.byref(desc)))


def mask_pack(desc: fmbym_mask_desc, stream) -> None:
    _check(lib().fmbym_mask_pack(ctypes.byref(desc), stream), "fmbym_mask_pack")


def mask_activation_bytes(desc, images: int, n: int) -> int:
    return int(lib().fmbym_mask_activation_bytes(ctypes.byref(desc), int(images), int(n)))


def mask_workspace_bytes(desc, images: int, n: int) -> int:
    return int(lib().fmbym_mask_workspace_bytes(ctypes.byref(desc), int(images), int(n)))


def mask_fwd(desc, images, n, x, mask, act, act_bytes, training, stream) -> None:
    _check(lib().fmbym_mask_fwd(ctypes.byref(desc), int(images), int(n), x, mask, act, int(act_bytes),
                                int(bool(training)), stream), "fmbym_mask_fwd")


def mask_bwd(desc, images, n, d_mask, act, act_bytes, d_params, ws, ws_bytes, stream, d_x=None) -> None:
    _check(lib().fmbym_mask_bwd(ctypes.byref(desc), int(images), int(n), d_mask, act, int(act_bytes),
                                d_params, d_x, ws, int(ws_bytes), stream), "fmbym_mask_bwd")


def adam(params, grad, m, v, count, step, lr, beta1, beta2, eps, stream) -> None:
    _check(lib().fmbym_adam(params, grad, m, v, int(count), int(step), float(lr), float(beta1),
                            float(beta2), float(eps), stream), "fmbym_adam")


def pose_loss(batch, pose, target, kind, loss, d_pose, stream) -> None:
    _check(lib().fmbym_pose_loss(int(batch), pose, target, int(kind), loss, d_pose, stream),
           "fmbym_pose_loss")


class MaskNet:
    """Device buffers of the mask network (FP32 parameters, BF16 packed
    weights, running statistics, Adam moments) and its calls on torch tensors.
    ``params`` uses the library's flat layout (include/fmbym_mask.h).
    channels = 2 is the dual-input network: scans and masks are passed as the
    stacked planes [f batch; g batch] ([2 B, n, n])."""

    def __init__(self, params, levels: int = 4, base: int = 8, bn_eps: float = 1e-5,
                 bn_momentum: float = 0.1, device="cuda:0", channels: int = 1):
        self.levels, self.base, self.channels = levels, base, channels
        self.desc = fmbym_mask_desc(levels, base, bn_eps, bn_momentum, None, None, None, channels)
        n_p = mask_param_count(self.desc)
        if n_p == 0:
            raise FmbymError(FMBYM_EUNSUPPORTED, "fmbym_mask_param_count")
        p = torch.as_tensor(params, dtype=torch.float32).to(device).contiguous()
        if p.numel() != n_p:
            raise ValueError(f"params: expected {n_p} values, got {p.numel()}")
        self.params = p
        self.packed = torch.zeros(mask_packed_bytes(self.desc), dtype=torch.uint8, device=device)
        nbn = mask_bn_channels(self.desc)
        self.bn_running = torch.cat([torch.zeros(nbn), torch.ones(nbn)]).to(device)
        self.m = torch.zeros_like(p)
        self.v = torch.zeros_like(p)
        self.step = 0
        self.desc.params = p.data_ptr()
        self.desc.packed = self.packed.data_ptr()
        self.desc.bn_running = self.bn_running.data_ptr()
        self._act = None
        self._ws = None
        self.pack()

    def pack(self) -> None:
        mask_pack(self.desc, _stream())

    def _buf(self, name, need, dev):
        cur = getattr(self, name)
        if cur is None or cur.numel() < need:
            cur = torch.empty(need, dtype=torch.uint8, device=dev)
            setattr(self, name, cur)
        return cur

    def forward(self, x, training: bool = True):
        """x [C I, n, n] float32 scans (C planes of I) -> masks [C I, n, n]; keeps the
        activations for backward."""
        C = self.channels
        I, n = x.shape[0] // C, x.shape[-1]
        if I * C != x.shape[0]:
            raise ValueError(f"x: {x.shape[0]} scans is not a multiple of {C} planes")
        need = mask_activation_bytes(self.desc, I, n)
        if need == 0:
            raise FmbymError(FMBYM_EUNSUPPORTED, "fmbym_mask_activation_bytes")
        act = self._buf("_act", need, x.device)
        mask = torch.empty(C * I, n, n, device=x.device)
        mask_fwd(self.desc, I, n, _ptr(x, (C * I, n, n), "x"), mask.data_ptr(), act.data_ptr(), act.numel(),
                 training, _stream())
        self._shape = (I, n)
        return mask

    def backward(self, d_mask, input_grad: bool = False):
        """dL/dparams (flat FP32) of the last training forward, given dL/dmask;
        with input_grad, the pair (dL/dparams, dL/dx)."""
        I, n = self._shape
        C = self.channels
        need = mask_workspace_bytes(self.desc, I, n)
        ws = self._buf("_ws", need, d_mask.device)
        d_params = torch.empty_like(self.params)
        d_x = torch.empty(C * I, n, n, device=d_mask.device) if input_grad else None
        mask_bwd(self.desc, I, n, _ptr(d_mask.contiguous(), (C * I, n, n), "d_mask"), self._act.data_ptr(),
                 self._act.numel(), d_params.data_ptr(), ws.data_ptr(), ws.numel(), _stream(),
                 d_x=None if d_x is None else d_x.data_ptr())
        return (d_params, d_x) if input_grad else d_params

    def adam_step(self, grad, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
        """One Adam update of params with grad, then re-pack the BF16 weights."""
        self.step += 1
        adam(self.params.data_ptr(), _ptr(grad.contiguous(), name="grad"), self.m.data_ptr(),
             self.v.data_ptr(), self.params.numel(), self.step, lr, beta1, beta2, eps, _stream())
        self.pack()


def pose_loss_t(pose, target, kind: int = FMBYM_LOSS_L2):
    """(loss [1], d_pose [B, 3]) on device tensors through fmbym_pose_loss."""
    B = pose.shape[0]
    loss = torch.empty(1, device=pose.device)
    d = torch.empty(B, 3, device=pose.device)
    pose_loss(B, _ptr(pose.contiguous(), (B, 3), "pose"), _ptr(target.contiguous(), (B, 3), "target"),
              kind, loss.data_ptr(), d.data_ptr(), _stream())
    return loss, d
