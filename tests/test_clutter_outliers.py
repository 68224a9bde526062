"""Why the squared pose loss trains less steadily than Eq. 13's L1 on the
mask-training scenes: the unmasked search's heading errors there are heavy
tailed, and the tail comes from the moving clutter blobs.

1. Mechanism.  The magnitude spectrum of a set of blobs is the blob envelope
   times |sum_k a_k exp(-i k.x_k)|: fringes perpendicular to each blob-to-blob
   offset, at low frequency where the envelope is largest.  The blobs move
   independently of the pose between the two scans, so their offsets turn by an
   angle that has nothing to do with the heading, and stage 1 (Eq. 5-8) follows
   the fringes: two blobs whose offset turns by phi give a heading of phi.
   The blobs' own correlation peaks pull the translation the same way.
2. With the blobs in the scene, 12 of the first 40 training pairs come out more
   than 20 degrees or 2 m off (7 in heading); with the same scenes and the
   blobs' amplitude set to zero, 2 do (none in heading).
3. Those pairs carry the squared loss: a pair metres off contributes tens of
   m^2 against ~0.05 for a good pair, so a few of them hold most of the L2 loss
   of a batch (and, through it, most of its gradient), far more than they hold
   of the L1 loss."""
import math

import numpy as np

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import synth, workloads

KW = workloads.search_kwargs("batch256")


def test_the_heading_follows_the_turn_of_a_blob_pair():
    p = O.Params(**KW)
    n, nth = KW["n"], KW["n_theta"]
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)

    def blobs(pts, sig=6.0):
        return sum(np.exp(-((xx - x) ** 2 + (yy - y) ** 2) / (2 * sig * sig)) for x, y in pts)

    d = np.array([30.0, 8.0])
    for phi in (40.0, -25.0, 70.0):
        c, s = math.cos(math.radians(phi)), math.sin(math.radians(phi))
        rd = np.array([c * d[0] - s * d[1], s * d[0] + c * d[1]])
        f = blobs([(100, 120), (100 + d[0], 120 + d[1])])
        g = blobs([(140, 100), (140 + rd[0], 100 + rd[1])])      # offset turned by phi, elsewhere
        c_theta = O.search(f, g, p)["c_theta"].numpy()
        lag = int(np.argmax(c_theta)) - nth // 2
        assert abs(lag - phi / (180.0 / nth)) <= 1.0, (phi, lag)


def _pose_errors(count, blob_scale):
    spec, wid = synth.WORKLOADS["mask256"], synth.WORKLOAD_ID["mask256"]
    p = O.Params(**KW)
    out = []
    for i in range(count):
        f, g, pose = synth.make_pair(spec, wid, "train", i, blob_scale=blob_scale)
        r = O.search(f, g, p)
        out.append(r["pose"].numpy() - pose)
    return np.array(out)


def test_clutter_blobs_cause_the_outliers_and_they_hold_the_squared_loss():
    count = 40
    with_blobs = _pose_errors(count, 1.0)
    without = _pose_errors(count, 0.0)

    def outliers(e):
        heading = np.abs(e[:, 0]) > math.radians(20.0)
        return heading, heading | (np.hypot(e[:, 1], e[:, 2]) > 2.0)

    h_with, o_with = outliers(with_blobs)
    h_without, o_without = outliers(without)
    print(f"pose off by > 20 deg or > 2 m: {o_with.sum()} of {count} with blobs ({h_with.sum()} in heading), "
          f"{o_without.sum()} without ({h_without.sum()} in heading)")
    assert h_with.sum() >= 5 and h_without.sum() == 0
    assert o_with.sum() >= 8 and o_without.sum() <= 2
    # the tenth of the pairs with the largest loss: their share of the batch's L2 and L1 loss
    l2 = (with_blobs ** 2).sum(1)
    l1 = np.abs(with_blobs).sum(1)
    k = count // 10
    share_l2 = np.sort(l2)[::-1][:k].sum() / l2.sum()
    share_l1 = np.sort(l1)[::-1][:k].sum() / l1.sum()
    print(f"largest tenth: {share_l2:.2f} of the L2 loss, {share_l1:.2f} of the L1 loss")
    assert share_l2 > 0.5 and share_l2 > share_l1 + 0.1
