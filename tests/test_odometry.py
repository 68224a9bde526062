"""Odometry host logic: chaining pair poses into a trajectory, the segment
drift metric, and the drive generator's pose convention (CPU only).

The metric is pinned on trajectories whose errors have closed forms; the
chaining on the generator's own world-frame poses; and the convention that
joins them on the oracle's search of rendered consecutive scans."""
import math

import numpy as np
import pytest

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import odometry, synth


def _straight(k, d):
    """k frames along +x, d metres apart, heading 0."""
    return np.stack([np.arange(k) * d, np.zeros(k), np.zeros(k)], axis=1)


def test_chaining_the_generated_pair_poses_gives_the_drive():
    """The generator derives each pair pose from world-frame vehicle poses;
    chaining them must rebuild those poses."""
    _, poses, rel = synth.make_drive("drive512", scans=False)
    np.testing.assert_allclose(odometry.chain(rel), poses, atol=1e-9)


def test_perfect_estimate_has_no_drift():
    _, poses, _ = synth.make_drive("drive512", scans=False)
    e = odometry.segment_errors(poses, poses)
    assert e["segments"] > 0 and e["t_pct"] == 0.0 and e["r_deg_per_km"] == 0.0
    assert sorted(e["per_length"]) == list(odometry.KITTI_LENGTHS_M)   # about 1 km: every length present


def test_scale_error_is_the_translational_drift():
    """Every pair translation 10 % too long on a straight path: the error of a
    segment is 10 % of the distance it spans, m d with m = floor(L / d) + 1
    pairs (it ends at the first frame strictly past L), over L; no rotational
    error."""
    gt = _straight(201, 2.5)
    rel = np.zeros((200, 3))
    rel[:, 1] = -2.5 * 1.1          # the world moves back by the step in the new frame
    est = odometry.chain(rel)
    np.testing.assert_allclose(odometry.chain(np.column_stack([np.zeros(200), -2.5 * np.ones(200),
                                                               np.zeros(200)])), gt, atol=1e-12)
    e = odometry.segment_errors(gt, est, lengths=(100, 200))
    assert e["r_deg_per_km"] == 0.0
    for L in (100, 200):
        m = math.floor(L / 2.5) + 1
        assert abs(e["per_length"][L][0] - 10.0 * m * 2.5 / L) < 1e-9


def test_heading_bias_is_the_rotational_drift():
    """A constant heading bias b per pair: over a segment of m pairs the
    rotation error is m b, with m = floor(L / d) + 1 on a path of steps d
    (the segment ends at the first frame strictly past L)."""
    d, b = 2.5, math.radians(0.01)
    gt = _straight(401, d)
    rel = np.zeros((400, 3))
    rel[:, 0] = b
    rel[:, 1] = -d
    est = odometry.chain(rel)
    for L in (100, 300):
        e = odometry.segment_errors(gt, est, lengths=(L,))
        m = math.floor(L / d) + 1
        assert abs(e["r_deg_per_km"] - math.degrees(m * b / L) * 1000.0) < 1e-9
        # chaining turns the whole path: the segment's end moves sideways, so translation drifts too
        assert e["t_pct"] > 0


@pytest.mark.slow
def test_drive_pairs_follow_the_search_convention():
    """The oracle's search of consecutive rendered scans returns the
    generator's pair poses (heading within a bin, translation within pixels),
    so chained search poses and the true drive share one convention."""
    scans, _, rel = synth.make_drive("drive256")
    p = O.Params(n=256, n_theta=256, delta_xy=0.35, band_lo=0.02, band_hi=0.4, temp_xy=0.05)
    for k in (0, 60):
        est = O.search(scans[k], scans[k + 1], p)["pose"].numpy()
        assert abs(est[0] - rel[k, 0]) <= math.pi / 256, (k, est, rel[k])
        assert math.hypot(est[1] - rel[k, 1], est[2] - rel[k, 2]) <= 3 * 0.35, (k, est, rel[k])


def test_outlier_gate_keeps_the_generated_motion():
    """The generator turns by a damped random walk of at most a few degrees
    per frame at 2-3 m per frame: no true pair pose breaks the gate."""
    for name in ("drive256", "drive512"):
        _, _, rel = synth.make_drive(name, scans=False)
        gated, rejected = odometry.gate_outliers(rel)
        assert not rejected.any()
        np.testing.assert_array_equal(gated, rel)


def test_outlier_gate_replaces_exactly_the_planted_outliers():
    """Pairs sent to a spurious heading peak (tens of degrees off, their
    translation metres off) are replaced, including the first pair and two in
    a row; the gated trajectory's drift falls back near the true one's."""
    _, gt, rel = synth.make_drive("drive512", scans=False)
    bad = [0, 37, 38, 150, 260, 399]
    est = rel.copy()
    for j, k in enumerate(bad):
        est[k, 0] += math.radians(25.0 if j % 2 == 0 else -40.0)
        est[k, 1] += 4.0
        est[k, 2] -= 3.0
    gated, rejected = odometry.gate_outliers(est)
    assert np.nonzero(rejected)[0].tolist() == bad
    keep = np.setdiff1d(np.arange(len(rel)), bad)
    np.testing.assert_array_equal(gated[keep], est[keep])
    # a replaced pair takes the median of its neighbours' motion
    assert np.abs(gated[bad, 0] - rel[bad, 0]).max() < math.radians(6.0)
    assert np.hypot(*(gated[bad, 1:] - rel[bad, 1:]).T).max() < 1.0
    raw = odometry.segment_errors(gt, odometry.chain(est))
    fixed = odometry.segment_errors(gt, odometry.chain(gated))
    assert fixed["t_pct"] < 0.2 * raw["t_pct"] and fixed["r_deg_per_km"] < 0.2 * raw["r_deg_per_km"]


def test_outlier_gate_follows_a_real_change_of_motion():
    """A step change of the motion lasting longer than max_run pairs is
    rejected max_run times, then accepted and followed."""
    rel = np.tile([0.0, -2.5, 0.0], (30, 1))
    rel[10:, 0] = math.radians(15.0)
    gated, rejected = odometry.gate_outliers(rel, max_run=3)
    assert np.nonzero(rejected)[0].tolist() == [10, 11, 12]
    np.testing.assert_array_equal(gated[13:], rel[13:])


def test_outlier_gate_on_short_and_empty_lists():
    """Fewer pairs than the prior's window, and none at all."""
    gated, rejected = odometry.gate_outliers(np.zeros((0, 3)))
    assert gated.shape == (0, 3) and rejected.shape == (0,)
    rel = np.array([[0.0, -2.5, 0.0], [0.0, -2.4, 0.1], [math.radians(30.0), 2.0, 0.0]])
    gated, rejected = odometry.gate_outliers(rel)
    assert rejected.tolist() == [False, False, True]
    np.testing.assert_array_equal(gated[2], np.median(rel, axis=0))
