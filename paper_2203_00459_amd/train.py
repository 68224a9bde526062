"""Training of the mask network through the differentiable search (Section III-E).

One step (Eq. 10-13): masks m = h_alpha(scan) for both scans of every pair
(one batched network call, shared weights), the search on the masked scans
(the training forward, which keeps its intermediates for the adjoint),
the pose loss against the known poses, the search's adjoint down to the masks,
the network's adjoint down to its parameters, and an Adam update.  Every
stage runs in the library's kernels; this module only sequences the calls.

The unmasked search is the fallback and the yardstick: ``evaluate`` reports the
pose error of both searches on held-out pairs, and ``use_mask`` is only set
once the masked search has beaten the unmasked one there.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
import torch

from . import fmbym


def he_init(levels: int, base: int, seed: int, channels: int = 1) -> np.ndarray:
    """Flat parameters in the library's layout: He-normal conv weights
    (std sqrt(2 / (9 c_in))), BatchNorm gamma 1 and beta 0, head weights with
    std sqrt(1 / (9 base)) and zero biases; `channels` scans in and masks out."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ch = [base << l for l in range(levels)]
    convs = []
    for l in range(levels):
        convs += [(channels if l == 0 else ch[l - 1], ch[l]), (ch[l], ch[l])]
    for l in range(levels - 2, -1, -1):
        convs += [(ch[l + 1] + ch[l], ch[l]), (ch[l], ch[l])]
    parts = []
    for cin, cout in convs:
        parts += [rng.normal(0.0, math.sqrt(2.0 / (9 * cin)), cout * cin * 9), np.ones(cout),
                  np.zeros(cout)]
    parts += [rng.normal(0.0, math.sqrt(1.0 / (9 * base)), channels * base * 9), np.zeros(channels)]
    return np.concatenate(parts).astype(np.float32)


@dataclasses.dataclass
class TrainConfig:
    levels: int = 4
    base: int = 8
    channels: int = 1          # 2: the dual-input network (both scans in, both masks out)
    lr: float = 1e-3
    loss: int = fmbym.FMBYM_LOSS_L2
    seed: int = 0


class MaskedSearchTrainer:
    """Mask network + masked search + loss + adjoints + Adam on one GPU."""

    def __init__(self, search_kwargs: dict, batch: int, cfg: TrainConfig = TrainConfig(),
                 params: np.ndarray | None = None):
        self.cfg = cfg
        self.batch = batch
        self.search = fmbym.Search(max_batch=batch, **search_kwargs)
        p = he_init(cfg.levels, cfg.base, cfg.seed, cfg.channels) if params is None else params
        self.net = fmbym.MaskNet(p, levels=cfg.levels, base=cfg.base, channels=cfg.channels)
        self.use_mask = False

    def masks(self, f, g, training: bool):
        """Masks of both scans of every pair: the scans stacked [f; g] go through
        the network as 2B images (shared weights) or, for the dual-input network,
        as B samples of two channels; either way the masks come back [m_f; m_g]."""
        B = f.shape[0]
        m = self.net.forward(torch.cat([f, g]), training=training)
        return m[:B].contiguous(), m[B:].contiguous()

    def step(self, f, g, target):
        """One training step on device tensors f, g [B, n, n] and target [B, 3];
        returns (loss tensor [1], pose [B, 3])."""
        m_f, m_g = self.masks(f, g, training=True)
        out = self.search.forward(f, g, m_f, m_g, keep=True)
        loss, d_pose = fmbym.pose_loss_t(out["pose"], target, self.cfg.loss)
        gr = self.search.backward(f, g, m_f, m_g, out, d_pose)
        d_params = self.net.backward(torch.cat([gr["d_m_f"], gr["d_m_g"]]))
        self.net.adam_step(d_params, self.cfg.lr)
        return loss, out["pose"]

    def gradient(self, f, g, target):
        """dL/dparams of the chain without updating (for checks)."""
        m_f, m_g = self.masks(f, g, training=True)
        out = self.search.forward(f, g, m_f, m_g, keep=True)
        loss, d_pose = fmbym.pose_loss_t(out["pose"], target, self.cfg.loss)
        gr = self.search.backward(f, g, m_f, m_g, out, d_pose)
        return loss, self.net.backward(torch.cat([gr["d_m_f"], gr["d_m_g"]]))

    @torch.no_grad()
    def evaluate(self, f, g, target) -> dict:
        """Mean |theta| error (rad) and mean translation error (m) of the masked
        (network in inference mode) and the unmasked search; sets use_mask."""
        m_f, m_g = self.masks(f, g, training=False)
        pm = self.search.forward(f, g, m_f, m_g, surfaces=False)["pose"]
        pu = self.search.forward(f, g, surfaces=False)["pose"]

        def err(p):
            d = (p - target).double()
            return float(d[:, 0].abs().mean()), float(d[:, 1:].norm(dim=1).mean())

        em, eu = err(pm), err(pu)
        # the comparison: translation error first (the paper's drift metric), heading as a tie-break
        self.use_mask = (em[1], em[0]) < (eu[1], eu[0])
        return {"masked_theta": em[0], "masked_t": em[1], "unmasked_theta": eu[0], "unmasked_t": eu[1],
                "use_mask": self.use_mask}

    # ------------------------------------------------------ checkpoint / resume

    def state_dict(self) -> dict:
        """Everything a resumed run needs, as CPU tensors and plain values: the
        FP32 master weights, Adam's moments and step count, the BatchNorm running
        statistics, the fallback decision and the configuration."""
        n = self.net
        return {"params": n.params.detach().cpu().clone(), "adam_m": n.m.cpu().clone(),
                "adam_v": n.v.cpu().clone(), "adam_step": int(n.step), "bn_running": n.bn_running.cpu().clone(),
                "use_mask": bool(self.use_mask), "config": dataclasses.asdict(self.cfg)}

    def load_state_dict(self, st: dict) -> None:
        """Restore a state_dict (in place: the device buffers keep their
        addresses) and re-pack the BF16 weights."""
        check_state(st, self.net.params.numel(), self.net.bn_running.numel())
        if st["config"]["levels"] != self.cfg.levels or st["config"]["base"] != self.cfg.base:
            raise ValueError("checkpoint of a different network")
        n = self.net
        n.params.copy_(st["params"].to(n.params.device))
        n.m.copy_(st["adam_m"].to(n.m.device))
        n.v.copy_(st["adam_v"].to(n.v.device))
        n.bn_running.copy_(st["bn_running"].to(n.bn_running.device))
        n.step = int(st["adam_step"])
        self.use_mask = bool(st["use_mask"])
        n.pack()

    def save(self, path: str, extra: dict | None = None) -> None:
        """Write the state (plus the caller's own plain values, e.g. its data
        order's RNG state, under "extra") with torch.save."""
        save_checkpoint(path, self.state_dict(), extra)

    def load(self, path: str) -> dict:
        """Restore from save(); returns the caller's "extra" values."""
        st = load_checkpoint(path)
        self.load_state_dict(st)
        return st.get("extra", {})

    @torch.no_grad()
    def predict(self, f, g, min_mask_mean: float = 1e-3):
        """Poses with the policy: the masked search once it has won, else the
        unmasked one; and per pair, the unmasked pose wherever the network has
        all but blanked a scan (mask mean below min_mask_mean)."""
        if not self.use_mask:
            return self.search.forward(f, g, surfaces=False)["pose"]
        m_f, m_g = self.masks(f, g, training=False)
        masked = self.search.forward(f, g, m_f, m_g, surfaces=False)["pose"]
        blank = blank_masks(m_f.mean(dim=(1, 2)), m_g.mean(dim=(1, 2)), min_mask_mean)
        if not bool(blank.any()):
            return masked
        plain = self.search.forward(f, g, surfaces=False)["pose"]
        return fallback_poses(masked, plain, blank)


def blank_masks(mean_f, mean_g, min_mean: float):
    """Pairs whose mask of either scan has a mean below min_mean [B] bool."""
    return (mean_f < min_mean) | (mean_g < min_mean)


def fallback_poses(masked, plain, blank):
    """The masked poses, with the unmasked pose in the rows flagged blank."""
    return torch.where(blank[:, None], plain, masked)


def check_state(st: dict, n_params: int, n_bn: int) -> None:
    """Shapes and types of a trainer state; raises ValueError on a mismatch."""
    for k in ("params", "adam_m", "adam_v"):
        if not isinstance(st.get(k), torch.Tensor) or st[k].numel() != n_params or st[k].dtype != torch.float32:
            raise ValueError(f"checkpoint field {k}: expected {n_params} float32 values")
    if not isinstance(st.get("bn_running"), torch.Tensor) or st["bn_running"].numel() != n_bn:
        raise ValueError(f"checkpoint field bn_running: expected {n_bn} values")
    if int(st.get("adam_step", -1)) < 0:
        raise ValueError("checkpoint field adam_step missing")


def save_checkpoint(path: str, state: dict, extra: dict | None = None) -> None:
    """torch.save of a trainer state (tensors and plain values only)."""
    st = dict(state)
    if extra is not None:
        st["extra"] = dict(extra)
    torch.save(st, path)


def load_checkpoint(path: str) -> dict:
    """torch.load with weights_only=True: tensors and plain values, no code."""
    return torch.load(path, map_location="cpu", weights_only=True)
