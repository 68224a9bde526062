"""Search parameter sets of the measured workloads (plain numbers, no arithmetic).

Each entry pairs a scene family of ``synth.WORKLOADS`` with ScanMatch's
parameters (Algorithm 1).  The band-pass is a hard annulus in cycles per pixel;
its cut-offs are not given by the method and are a reading of this library.
"""

SEARCH = {
    # one pair, 128 x 128, 128 angle bins, both temperatures 1, forward only
    "pair128": dict(batch=1, n=128, n_theta=128, delta_xy=0.5, temp_theta=1.0, temp_xy=1.0,
                    band_lo=0.02, band_hi=0.40),
    # 64 pairs, 256 x 256, 256 angle bins
    "batch256": dict(batch=64, n=256, n_theta=256, delta_xy=0.35, temp_theta=1.0, temp_xy=1.0,
                     band_lo=0.02, band_hi=0.40),
    # 32 pairs, 512 x 512, 512 angle bins, forward and adjoint (the headline workload)
    "batch512": dict(batch=32, n=512, n_theta=512, delta_xy=0.2, temp_theta=1.0, temp_xy=1.0,
                     band_lo=0.02, band_hi=0.40),
    # the paper's measured sizes and ScanMatch defaults: 733 heading bins, T_theta = 2, T_xy = 1;
    # 32 pairs per batch, forward
    "paper127": dict(batch=32, n=127, n_theta=733, delta_xy=0.8, temp_theta=2.0, temp_xy=1.0,
                     band_lo=0.02, band_hi=0.40),
    "paper255": dict(batch=32, n=255, n_theta=733, delta_xy=0.4, temp_theta=2.0, temp_xy=1.0,
                     band_lo=0.02, band_hi=0.40),
    "paper511": dict(batch=32, n=511, n_theta=733, delta_xy=0.2, temp_theta=2.0, temp_xy=1.0,
                     band_lo=0.02, band_hi=0.40),
}

# What one bench step of each search workload runs: the forward alone (one pair,
# timed as a captured launch), the forward beside the joint comparator over
# 64 headings, or the forward and the adjoint.
PASS = {"pair128": "fwd", "batch256": "fwd+joint64", "batch512": "fwd+bwd",
        "paper127": "fwd", "paper255": "fwd", "paper511": "fwd"}
JOINT_ANGLES = 64

# Ragged serving batches: pairs of the three sizes above in one launch.
RAGGED = {
    # 1024 pairs: half 128 x 128, 30 % 256 x 256, 20 % 512 x 512, each with its size's parameters
    "ragged1024": dict(n_pairs=1024, mix=(("pair128", 0.5), ("batch256", 0.3), ("batch512", 0.2))),
    # the same list with every pair masked by the 4-level mask network inside the launch
    "ragged1024_masked": dict(n_pairs=1024, mix=(("pair128", 0.5), ("batch256", 0.3), ("batch512", 0.2)),
                              mask="net"),
}

# Mask-network training: batch of pairs with distractors, the 4-level network.
TRAIN = {
    # 16 pairs of 256 x 256 scans with moving clutter and multipath ghosts; search as batch256
    "mask256": dict(batch=16, n=256, levels=4, scenes="mask256", search="batch256"),
    # Table II's dual-input network (6 levels, 8 -> 256 channels, both scans in, both
    # masks out) at 512 x 512 with distractors, 4 pairs per step, L1 loss (Eq. 13),
    # Adam at 1e-4; search as batch512
    "dual512": dict(batch=4, n=512, levels=6, channels=2, scenes="mask512", search="batch512", loss="l1"),
}


# Mask-network inference on the running statistics, the pass the masked ragged
# launch runs: both scans of each pair through the 4-level network.
INFER = {
    # 32 pairs of 512 x 512 scans with distractors: 64 images
    "mask512_infer": dict(pairs=32, n=512, levels=4, scenes="mask512"),
}


# The configured mask-learning run: a fixed training set, trained for whole
# epochs under each loss from the same initialisation and data order, judged on
# held-out pairs against the unmasked search.
TRAIN_RUN = {
    # 20,000 pairs of 256 x 256 scans with distractors, batch 16, two epochs at
    # Adam 1e-3; the squared pose loss, with Eq. 13's L1 beside it
    "mask256_20k": dict(pairs=20000, held_out=256, batch=16, epochs=2, lr=1e-3, levels=4,
                        scenes="mask256", search="batch256", losses=("l2", "l1")),
}


# Radar odometry: the forward search over every consecutive pair of a drive
# (synth.DRIVES), all pairs in one launch, chained and scored over segments.
DRIVE = {
    # 401 frames at 512 x 512 (about 1 km): 400 pairs with batch512's parameters
    "drive512": dict(drive="drive512", search="batch512"),
}


def search_kwargs(name: str) -> dict:
    """Keyword arguments shared by the library's Search and the oracle's Params."""
    d = dict(SEARCH[name])
    d.pop("batch")
    return d
