"""Radar odometry on the GPU: the forward search over every consecutive pair
of a drive in one call (f = scans[:-1], g = scans[1:], overlapping views of
one array), chained into a trajectory and scored over segments.

Parity: sampled pairs against the oracle at the forward's bar (1e-3 rad,
1e-3 px), and the overlapping views give exactly the poses of separate
copies.  The accuracy bounds are a regression guard on this generated drive,
not a parity claim: per pair, the heading is within two bins and the
translation within two pixels on most pairs; the method also has outliers
(a spurious angular peak sends a pair tens of degrees off, and its
translation with it), which is what the chained trajectory's drift
mostly measures, so the drift bound is loose."""
import math

import numpy as np
import pytest
import torch

from oracle import fmbym_oracle as O
from paper_2203_00459_amd import fmbym, odometry, synth, workloads

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def test_drive_odometry_matches_the_oracle():
    scans, gt, rel = synth.make_drive("drive256")
    kw = workloads.search_kwargs("batch256")
    S = torch.from_numpy(scans).to(DEV)
    P = len(scans) - 1
    s = fmbym.Search(max_batch=P, **kw)
    est = s.forward(S[:-1], S[1:], surfaces=False)["pose"]
    copies = s.forward(S[:-1].clone(), S[1:].clone(), surfaces=False)["pose"]
    torch.cuda.synchronize()
    assert torch.equal(est, copies)
    est = est.double().cpu().numpy()
    s.close()
    p = O.Params(**kw)
    for k in (0, 57, P - 1):
        ref = O.search(scans[k], scans[k + 1], p)["pose"].numpy()
        d_th = abs(est[k, 0] - ref[0])
        d_t = max(abs(est[k, 1] - ref[1]), abs(est[k, 2] - ref[2])) / kw["delta_xy"]
        print(f"pair {k}: dtheta {d_th:.2e} rad dt {d_t:.2e} px", flush=True)
        assert d_th <= 1e-3 and d_t <= 1e-3
    traj = odometry.chain(est)
    e = odometry.segment_errors(gt, traj, lengths=(50, 100, 200))
    step_err = np.hypot(*(est[:, 1:] - rel[:, 1:]).T)
    print(f"drift {e['t_pct']:.2f} % {e['r_deg_per_km']:.1f} deg/km over {e['segments']} segments; "
          f"per pair: heading median {np.median(np.abs(est[:, 0] - rel[:, 0])):.4f} rad, "
          f"translation median {np.median(step_err):.3f} m; end point off by "
          f"{math.hypot(*(traj[-1, :2] - gt[-1, :2])):.2f} m after {len(gt)} frames; pairs within 2 bins "
          f"{(np.abs(est[:, 0] - rel[:, 0]) <= 2 * math.pi / kw['n_theta']).mean():.2f}", flush=True)
    gated, rejected = odometry.gate_outliers(est)
    eg = odometry.segment_errors(gt, odometry.chain(gated), lengths=(50, 100, 200))
    print(f"with the outlier gate: {int(rejected.sum())} pairs replaced, drift {eg['t_pct']:.2f} % "
          f"{eg['r_deg_per_km']:.1f} deg/km", flush=True)
    step = math.pi / kw["n_theta"]
    assert (np.abs(est[:, 0] - rel[:, 0]) <= 2 * step).mean() >= 0.85
    assert np.median(step_err) <= 2 * kw["delta_xy"]
    assert e["segments"] > 0
    assert e["t_pct"] <= 40.0 and e["r_deg_per_km"] <= 500.0
