"""Radar odometry from consecutive scan pairs: chaining the search's poses into
a trajectory, and the segment drift the paper reports (Table III(b): mean
translational error in percent and rotational error in degrees per kilometre
over segments of 100 ... 800 m, the KITTI odometry protocol).

Host arithmetic on a few hundred poses; no GPU code.  Poses of the trajectory
are (x, y, psi): the vehicle's pose in the world frame, a point y of the
scan's frame being the world point R(psi) y + (x, y).  Pair poses are the
search's (theta, t_x, t_y) for f = scan k, g = scan k + 1: a point at x in
frame k appears at R(theta) x + t in frame k + 1 (Eq. 1).
"""
from __future__ import annotations

import math

import numpy as np

KITTI_LENGTHS_M = (100, 200, 300, 400, 500, 600, 700, 800)


def _rot(a: float) -> np.ndarray:
    c, s = math.cos(a), math.sin(a)
    return np.array([[c, -s], [s, c]])


def chain(rel, start=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Trajectory [K, 3] from K - 1 pair poses [K - 1, 3].

    Frame k + 1 maps a frame-k point x to R(theta) x + t, so the vehicle turns
    by -theta and moves to p_k - R(psi_{k+1}) t."""
    rel = np.asarray(rel, dtype=np.float64)
    out = np.zeros((len(rel) + 1, 3))
    out[0] = start
    for k, (th, tx, ty) in enumerate(rel):
        psi = out[k, 2] - th
        out[k + 1, :2] = out[k, :2] - _rot(psi) @ np.array([tx, ty])
        out[k + 1, 2] = psi
    return out


def _between(a: np.ndarray, b: np.ndarray) -> tuple:
    """Pose of b in the frame of a: (dx, dy, dpsi)."""
    d = _rot(-a[2]) @ (b[:2] - a[:2])
    return d[0], d[1], b[2] - a[2]


def _wrap(a: float) -> float:
    return (a + math.pi) % (2 * math.pi) - math.pi


def segment_errors(gt, est, lengths=KITTI_LENGTHS_M, step: int = 10) -> dict:
    """Segment drift of an estimated trajectory against the true one.

    For every first frame i (every ``step``-th) and every length L, the
    segment ends at the first frame j whose distance along the true path from
    i exceeds L.  Its error is the pose of the estimated motion i -> j in the
    frame of the true motion i -> j: translational error |t_err| / L,
    rotational error |angle| / L.  Returns the means over all segments
    (``t_pct``: percent, ``r_deg_per_km``), the per-length means and the
    segment count; lengths the trajectory is too short for are left out."""
    gt = np.asarray(gt, dtype=np.float64)
    est = np.asarray(est, dtype=np.float64)
    step_len = np.hypot(*np.diff(gt[:, :2], axis=0).T)
    dist = np.concatenate([[0.0], np.cumsum(step_len)])
    t_all, r_all, per = [], [], {}
    for L in lengths:
        t_l, r_l = [], []
        for i in range(0, len(gt), step):
            js = np.nonzero(dist > dist[i] + L)[0]
            if len(js) == 0:
                break
            j = int(js[0])
            gx, gy, gp = _between(gt[i], gt[j])
            ex, ey, ep = _between(est[i], est[j])
            # error pose E = (true motion)^-1 (estimated motion)
            d = _rot(-gp) @ np.array([ex - gx, ey - gy])
            t_l.append(float(np.hypot(*d)) / L)
            r_l.append(abs(_wrap(ep - gp)) / L)
        if t_l:
            per[L] = (100.0 * float(np.mean(t_l)), math.degrees(float(np.mean(r_l))) * 1000.0, len(t_l))
            t_all += t_l
            r_all += r_l
    if not t_all:
        return dict(t_pct=None, r_deg_per_km=None, per_length=per, segments=0)
    return dict(t_pct=100.0 * float(np.mean(t_all)), r_deg_per_km=math.degrees(float(np.mean(r_all))) * 1000.0,
                per_length=per, segments=len(t_all))


def gate_outliers(rel, max_dtheta: float = math.radians(10.0), max_dt: float = 1.5, window: int = 5,
                  max_run: int = 10):
    """Replace pair poses that break a motion prior before chaining (an option:
    the paper chains the search's poses as they are).

    The prior of pair k is the component-wise median of the last ``window``
    accepted pair poses (at the start, of the first ``window`` pair poses): the
    vehicle's motion changes little between consecutive frames, while a pair
    whose heading went to a spurious angular peak is tens of degrees off, its
    translation with it.  A pair whose heading differs from the prior by more
    than ``max_dtheta`` (rad) or whose translation differs by more than
    ``max_dt`` (the pose's length unit) takes the prior's pose instead; after
    ``max_run`` rejections in a row (by default 10: 2.5 s of scans at 4 Hz) the next pair is
    accepted as it is and the prior starts again from it, so that a real change
    of motion is followed.  Returns (gated poses [K - 1, 3],
    rejected [K - 1] bool)."""
    rel = np.asarray(rel, dtype=np.float64)
    out = rel.copy()
    rejected = np.zeros(len(rel), dtype=bool)
    accepted = list(rel[:window])
    run = 0
    for k in range(len(rel)):
        prior = np.median(np.asarray(accepted[-window:]), axis=0)
        off = abs(_wrap(rel[k, 0] - prior[0])) > max_dtheta or math.hypot(*(rel[k, 1:] - prior[1:])) > max_dt
        if off and run < max_run:
            out[k] = prior
            rejected[k] = True
            run += 1
            continue
        if off:
            accepted = [rel[k]]          # the motion changed: the prior starts again from here
        elif k >= window:
            accepted.append(rel[k])
        run = 0
    return out, rejected
