"""Seeded synthetic radar-like scan pairs with a known SE(2) pose.

This module only draws inputs.  It contains none of the search's arithmetic
(no transforms, no correlation, no soft-argmax), so both the FP64 oracle and
the HIP path may consume its output.

Data model (Section III-A, Eq. 1): a world point at ``x`` in the frame of scan
``f`` appears at ``x' = R(theta*) x + t*`` in the frame of scan ``g``, so that
``f(x) ~= g(R x + t)``.  Pixel ``[i, j]`` of an ``n x n`` scan sits at
``x = (j - c) * delta`` and ``y = (i - c) * delta`` metres with ``c = n // 2``
(``n/2`` for even n, ``(n - 1)/2`` for odd n); the sensor is at pixel ``(c, c)``.

The real scans the method was evaluated on (a public FMCW radar dataset) are
not available, so these scenes stand in for them: non-negative power images
with point reflectors, line segments, a 1/r range falloff and Rayleigh
speckle, and inter-scan motion of a car at a 4 Hz scan rate
(|theta| <= 10 deg, |t| <= 3 m).  The distractor variant adds moving clutter
blobs and multipath ghosts, which do not follow the SE(2) motion and which a
learned mask should suppress (Section III-E).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class SceneSpec:
    """Recipe for one family of synthetic scan pairs."""

    n: int                      # scan side in pixels
    delta: float                # metres per pixel
    n_reflectors: int           # point reflectors, amplitude U[0.5, 1]
    n_segments: int             # line segments, amplitude U[0.3, 0.8]
    speckle_sigma: float        # Rayleigh speckle scale
    theta_max_deg: float = 10.0
    t_max_m: float = 3.0
    distractors: bool = False   # moving blobs + multipath ghosts
    falloff_m: float = 5.0      # returns are scaled by min(1, falloff_m / r)
    reflector_psf_px: float = 1.0
    segment_psf_px: float = 0.7


# Workloads, named by what they are.
WORKLOADS = {
    # one pair, 128 x 128 at 0.5 m/px, 40 reflectors, 10 segments, speckle 0.1
    "pair128": SceneSpec(n=128, delta=0.5, n_reflectors=40, n_segments=10, speckle_sigma=0.10),
    # batches at 256 x 256, 0.35 m/px, 60 reflectors, 20 segments, speckle 0.15
    "batch256": SceneSpec(n=256, delta=0.35, n_reflectors=60, n_segments=20, speckle_sigma=0.15),
    # batches at 512 x 512, 0.2 m/px (102.4 m field of view), same scene density
    "batch512": SceneSpec(n=512, delta=0.2, n_reflectors=60, n_segments=20, speckle_sigma=0.15),
    # the paper's three measured sizes (odd sides, about 102 m across each), c3's scene density
    "paper127": SceneSpec(n=127, delta=0.8, n_reflectors=60, n_segments=20, speckle_sigma=0.15),
    "paper255": SceneSpec(n=255, delta=0.4, n_reflectors=60, n_segments=20, speckle_sigma=0.15),
    "paper511": SceneSpec(n=511, delta=0.2, n_reflectors=60, n_segments=20, speckle_sigma=0.15),
    # mask-training pairs at 256 x 256 with moving clutter and multipath ghosts
    "mask256": SceneSpec(n=256, delta=0.35, n_reflectors=60, n_segments=20, speckle_sigma=0.15,
                         distractors=True),
    # the same at 512 x 512, 0.2 m/px (the dual-input network's training pairs)
    "mask512": SceneSpec(n=512, delta=0.2, n_reflectors=60, n_segments=20, speckle_sigma=0.15,
                         distractors=True),
}

# Seed stream of each family (fixed: adding a family never reseeds another).
WORKLOAD_ID = {"batch256": 1, "batch512": 2, "mask256": 3, "pair128": 4, "paper127": 5, "paper255": 6,
               "paper511": 7, "mask512": 8}

SPLIT_OFFSET = {"train": 0, "val": 1_000_000, "test": 2_000_000, "bench": 3_000_000}


def _rng(workload_id: int, split: str, index: int) -> np.random.Generator:
    key = [int(workload_id), SPLIT_OFFSET[split] + int(index)]
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(key)))


def _rot(theta: float) -> np.ndarray:
    c, s = math.cos(theta), math.sin(theta)
    return np.array([[c, -s], [s, c]])


def _to_px(p: np.ndarray, n: int, delta: float) -> np.ndarray:
    """World metres (x, y) -> fractional pixel (col, row)."""
    return p / delta + (n // 2)


def _splat_gaussian(img: np.ndarray, col: float, row: float, amp: float, sigma: float) -> None:
    n = img.shape[0]
    r = int(math.ceil(4 * sigma)) + 1
    i0, i1 = max(0, int(math.floor(row)) - r), min(n, int(math.floor(row)) + r + 2)
    j0, j1 = max(0, int(math.floor(col)) - r), min(n, int(math.floor(col)) + r + 2)
    if i0 >= i1 or j0 >= j1:
        return
    ii = np.arange(i0, i1)[:, None]
    jj = np.arange(j0, j1)[None, :]
    img[i0:i1, j0:j1] += amp * np.exp(-((ii - row) ** 2 + (jj - col) ** 2) / (2 * sigma * sigma))


def _splat_segment(img: np.ndarray, a: np.ndarray, b: np.ndarray, amp: float, sigma: float) -> None:
    """Gaussian tube around the segment a-b; a, b are (col, row) pixel coordinates."""
    n = img.shape[0]
    r = int(math.ceil(4 * sigma)) + 1
    i0 = max(0, int(math.floor(min(a[1], b[1]))) - r)
    i1 = min(n, int(math.floor(max(a[1], b[1]))) + r + 2)
    j0 = max(0, int(math.floor(min(a[0], b[0]))) - r)
    j1 = min(n, int(math.floor(max(a[0], b[0]))) + r + 2)
    if i0 >= i1 or j0 >= j1:
        return
    ii = np.arange(i0, i1)[:, None].astype(np.float64)
    jj = np.arange(j0, j1)[None, :].astype(np.float64)
    d = b - a
    L2 = float(d @ d)
    if L2 == 0.0:
        u = np.zeros_like(ii + jj)
    else:
        u = np.clip(((jj - a[0]) * d[0] + (ii - a[1]) * d[1]) / L2, 0.0, 1.0)
    dx = jj - (a[0] + u * d[0])
    dy = ii - (a[1] + u * d[1])
    img[i0:i1, j0:j1] += amp * np.exp(-(dx * dx + dy * dy) / (2 * sigma * sigma))


@dataclasses.dataclass
class _World:
    reflectors: np.ndarray      # [k, 2] metres
    refl_amp: np.ndarray        # [k]
    seg_a: np.ndarray           # [m, 2]
    seg_b: np.ndarray           # [m, 2]
    seg_amp: np.ndarray         # [m]


def _draw_world(spec: SceneSpec, rng: np.random.Generator) -> _World:
    radius = 0.45 * spec.n * spec.delta

    def disc(k):
        r = radius * np.sqrt(rng.uniform(0, 1, k))
        a = rng.uniform(0, 2 * np.pi, k)
        return np.stack([r * np.cos(a), r * np.sin(a)], axis=1)

    refl = disc(spec.n_reflectors)
    refl_amp = rng.uniform(0.5, 1.0, spec.n_reflectors)
    centre = disc(spec.n_segments)
    length = rng.uniform(2.0, 15.0, spec.n_segments)
    orient = rng.uniform(0, np.pi, spec.n_segments)
    half = 0.5 * length[:, None] * np.stack([np.cos(orient), np.sin(orient)], axis=1)
    seg_amp = rng.uniform(0.3, 0.8, spec.n_segments)
    return _World(refl, refl_amp, centre - half, centre + half, seg_amp)


def _render(spec: SceneSpec, world: _World, rot: np.ndarray, t: np.ndarray) -> np.ndarray:
    """Render the world as seen from a sensor whose frame maps x -> rot @ x + t."""
    n, delta = spec.n, spec.delta
    img = np.zeros((n, n), dtype=np.float64)
    for p, amp in zip(world.reflectors, world.refl_amp):
        q = _to_px(rot @ p + t, n, delta)
        _splat_gaussian(img, q[0], q[1], amp, spec.reflector_psf_px)
    for a, b, amp in zip(world.seg_a, world.seg_b, world.seg_amp):
        _splat_segment(img, _to_px(rot @ a + t, n, delta), _to_px(rot @ b + t, n, delta), amp,
                       spec.segment_psf_px)
    return img


def _falloff(spec: SceneSpec) -> np.ndarray:
    n, delta = spec.n, spec.delta
    c = (np.arange(n) - n // 2) * delta
    r = np.sqrt(c[None, :] ** 2 + c[:, None] ** 2)
    with np.errstate(divide="ignore"):
        return np.minimum(1.0, np.where(r > 0, spec.falloff_m / np.maximum(r, 1e-12), 1.0))


def _distractors(spec: SceneSpec, world: _World, rng: np.random.Generator, img: np.ndarray,
                 rot: np.ndarray, t: np.ndarray, blobs: list) -> None:
    n, delta = spec.n, spec.delta
    # moving clutter blobs: drawn once per pair, displaced independently per scan
    for centre, sig_m, amp, shift in blobs:
        q = _to_px(rot @ centre + t + shift, n, delta)
        _splat_gaussian(img, q[0], q[1], amp, sig_m / delta)
    # multipath ghosts of the strongest reflectors, radially scaled about the sensor
    strongest = np.argsort(-world.refl_amp)[:5]
    for k in strongest:
        p = rot @ world.reflectors[k] + t
        q = _to_px(rng.uniform(1.3, 2.0) * p, n, delta)
        _splat_gaussian(img, q[0], q[1], world.refl_amp[k] * rng.uniform(0.3, 0.6),
                        spec.reflector_psf_px)


def make_pair(spec: SceneSpec, workload_id: int, split: str, index: int,
              theta: float | None = None, t: tuple[float, float] | None = None,
              blob_scale: float = 1.0):
    """Return (f, g, pose) with f, g float32 [n, n] and pose float64 (theta rad, tx m, ty m).

    ``blob_scale`` scales the clutter blobs' amplitude (0 removes them) without
    changing any random draw, so the rest of the pair is the same scene."""
    rng = _rng(workload_id, split, index)
    world = _draw_world(spec, rng)
    th = rng.uniform(-1, 1) * math.radians(spec.theta_max_deg)
    tt = rng.uniform(-spec.t_max_m, spec.t_max_m, 2)
    if theta is not None:
        th = float(theta)
    if t is not None:
        tt = np.asarray(t, dtype=np.float64)
    blobs = []
    if spec.distractors:
        radius = 0.4 * spec.n * spec.delta
        for _ in range(5):
            r = radius * math.sqrt(rng.uniform())
            a = rng.uniform(0, 2 * math.pi)
            blobs.append((np.array([r * math.cos(a), r * math.sin(a)]), rng.uniform(1.0, 3.0),
                          blob_scale * rng.uniform(0.5, 1.0), None))
    fall = _falloff(spec)
    scans = []
    for rot, tr in ((np.eye(2), np.zeros(2)), (_rot(th), tt)):
        img = _render(spec, world, rot, tr)
        if spec.distractors:
            shifted = [(c, s, a, rng.uniform(-5.0, 5.0, 2)) for (c, s, a, _) in blobs]
            _distractors(spec, world, rng, img, rot, tr, shifted)
        img *= fall
        img += rng.rayleigh(spec.speckle_sigma, img.shape)
        scans.append(img.astype(np.float32))
    return scans[0], scans[1], np.array([th, tt[0], tt[1]], dtype=np.float64)


def make_batch(name: str, batch: int, split: str = "test", start: int = 0,
               theta_max_deg: float | None = None):
    """Stack ``batch`` pairs of workload ``name``: f, g float32 [B, n, n]; pose float64 [B, 3].

    ``theta_max_deg`` widens the heading prior (180: headings over the whole
    circle, the metric-localisation case); the seeds are those of ``name``."""
    spec = WORKLOADS[name]
    if theta_max_deg is not None:
        spec = dataclasses.replace(spec, theta_max_deg=float(theta_max_deg))
    wid = WORKLOAD_ID[name]
    fs, gs, ps = [], [], []
    for i in range(batch):
        f, g, p = make_pair(spec, wid, split, start + i)
        fs.append(f)
        gs.append(g)
        ps.append(p)
    return np.stack(fs), np.stack(gs), np.stack(ps)


def _batch_chunk(args):
    name, split, start, count = args
    return start, make_batch(name, count, split=split, start=start)


def make_batch_parallel(name: str, batch: int, split: str = "train", workers: int | None = None,
                        chunk: int = 250):
    """``make_batch`` spread over worker processes: the same pairs in the same
    order (every pair has its own seed).  The workers are spawned, so this may
    be called from a process that already uses the GPU."""
    import multiprocessing as mp
    import os
    if workers is None:
        workers = min(16, os.cpu_count() or 1)
    spec = WORKLOADS[name]
    f = np.empty((batch, spec.n, spec.n), np.float32)
    g = np.empty_like(f)
    p = np.empty((batch, 3), np.float64)
    jobs = [(name, split, s, min(chunk, batch - s)) for s in range(0, batch, chunk)]
    with mp.get_context("spawn").Pool(workers) as pool:
        for start, (a, b, c) in pool.imap_unordered(_batch_chunk, jobs):
            f[start:start + len(a)], g[start:start + len(a)], p[start:start + len(a)] = a, b, c
    return f, g, p


def noise_batch(n: int, batch: int, seed: int = 0):
    """Uniform-noise scans, the input used for the method's timing runs (Section IV-C)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random((batch, n, n), dtype=np.float32), rng.random((batch, n, n), dtype=np.float32))


def ragged_mix(n_pairs: int, mix, seed: int = 0) -> list[str]:
    """Workload names for a ragged work list: ``mix`` is ((name, fraction), ...);
    counts are rounded down, the remainder goes to the first entry, and the
    order is a seeded shuffle."""
    counts = [int(math.floor(frac * n_pairs)) for _, frac in mix]
    counts[0] += n_pairs - sum(counts)
    names = [name for (name, _), c in zip(mix, counts) for _ in range(c)]
    rng = np.random.Generator(np.random.PCG64(seed))
    return [names[i] for i in rng.permutation(n_pairs)]


# ------------------------------------------------------------------ drives

@dataclasses.dataclass(frozen=True)
class DriveSpec:
    """A drive through a static world with one scan per frame: consecutive scans
    are the pairs of radar odometry (Section IV: scans at 4 Hz, poses chained
    into a trajectory and scored over segments, Table III(b))."""

    scene: str                          # WORKLOADS key: scan size, resolution, scene density
    frames: int
    step_m: tuple = (2.0, 3.0)          # distance driven per frame (about 10 m/s at 4 Hz)
    yaw_step_deg: float = 4.0           # bound of the per-frame heading change


DRIVES = {
    # 401 frames at 512 x 512, 0.2 m/px: about 1 km, long enough for segments of 100 ... 800 m
    "drive512": DriveSpec(scene="batch512", frames=401),
    # 121 frames at 256 x 256, 0.35 m/px: about 300 m
    "drive256": DriveSpec(scene="batch256", frames=121),
}


def make_drive(name: str, split: str = "test", index: int = 0, scans: bool = True):
    """Return (scans, poses, rel).

    scans  float32 [K, n, n], scan k seen from the vehicle at frame k (None if
           ``scans`` is False);
    poses  float64 [K, 3], the vehicle pose (x, y, psi) in the world frame,
           starting at (0, 0, 0): a point y of scan k's frame is the world
           point R(psi) y + (x, y);
    rel    float64 [K-1, 3], the pose (theta, t_x, t_y) of each consecutive
           pair f = scan k, g = scan k + 1 in ``make_pair``'s convention (a
           point at x in frame k appears at R(theta) x + t in frame k + 1):
           theta = psi_k - psi_{k+1}, t = R(-psi_{k+1}) (p_k - p_{k+1}).

    The world holds reflectors and segments at the single-pair scenes' density
    (their count per disc of radius 0.45 n delta), drawn over the drive's
    bounding box; every scan gets its own speckle.
    """
    ds = DRIVES[name]
    spec = WORKLOADS[ds.scene]
    rng = _rng(100 + sorted(DRIVES).index(name), split, index)
    K = ds.frames
    psi = np.zeros(K)
    pos = np.zeros((K, 2))
    rate = 0.0
    for k in range(1, K):
        # heading change per frame: a damped random walk, bounded
        rate = float(np.clip(0.8 * rate + rng.normal(0.0, 1.5), -ds.yaw_step_deg, ds.yaw_step_deg))
        psi[k] = psi[k - 1] + math.radians(rate)
        pos[k] = pos[k - 1] + rng.uniform(*ds.step_m) * np.array([math.cos(psi[k]), math.sin(psi[k])])
    rel = np.zeros((K - 1, 3))
    for k in range(K - 1):
        rel[k, 0] = psi[k] - psi[k + 1]
        rel[k, 1:] = _rot(-psi[k + 1]) @ (pos[k] - pos[k + 1])
    poses = np.concatenate([pos, psi[:, None]], axis=1)
    if not scans:
        return None, poses, rel
    # static world over the drive's bounding box (a scan sees objects up to its
    # half-diagonal away, plus half a segment)
    reach = (spec.n / 2) * spec.delta * math.sqrt(2.0) + 8.0
    lo, hi = pos.min(0) - reach, pos.max(0) + reach
    per_area = 1.0 / (math.pi * (0.45 * spec.n * spec.delta) ** 2)
    box = float(np.prod(hi - lo))
    n_refl = int(rng.poisson(spec.n_reflectors * box * per_area))
    n_seg = int(rng.poisson(spec.n_segments * box * per_area))
    refl = lo + (hi - lo) * rng.uniform(0.0, 1.0, (n_refl, 2))
    refl_amp = rng.uniform(0.5, 1.0, n_refl)
    centre = lo + (hi - lo) * rng.uniform(0.0, 1.0, (n_seg, 2))
    length = rng.uniform(2.0, 15.0, n_seg)
    orient = rng.uniform(0, np.pi, n_seg)
    half = 0.5 * length[:, None] * np.stack([np.cos(orient), np.sin(orient)], axis=1)
    seg_amp = rng.uniform(0.3, 0.8, n_seg)
    fall = _falloff(spec)
    out = np.empty((K, spec.n, spec.n), dtype=np.float32)
    for k in range(K):
        near_r = np.linalg.norm(refl - pos[k], axis=1) <= reach
        near_s = np.linalg.norm(centre - pos[k], axis=1) <= reach
        world = _World(refl[near_r], refl_amp[near_r], (centre - half)[near_s], (centre + half)[near_s],
                       seg_amp[near_s])
        rot = _rot(-psi[k])            # world -> frame k: y = R(-psi) (x - p)
        img = _render(spec, world, rot, -rot @ pos[k])
        img *= fall
        img += rng.rayleigh(spec.speckle_sigma, img.shape)
        out[k] = img.astype(np.float32)
    return out, poses, rel
