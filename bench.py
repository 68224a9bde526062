"""Throughput benchmark of the decoupled pose search on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch512]

One step is one pass of the search over one batch of synthetic scan pairs
already resident in HBM: the forward search and, when the adjoint is built,
its backward pass (fwd+bwd).  Prints one JSON line with the throughput in
scan pairs per second, a live roofline entry for the dominant kernel (its
per-launch algorithmic bytes over its average launch time, from HIP events
recorded around every library launch in a second timed pass), and the FP64
oracle timed on the host's cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, vendor figure
FP32_PEAK_TFLOPS = 157.3     # MI355X vector FP32, vendor figure
BF16_PEAK_TFLOPS = 2500.0    # MI355X dense BF16 matrix cores, vendor figure


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_batch512.txt")
# Table III(a), f-raw (the decoupled search without a mask), Hz at batch 1:
# (ThinkPad i7 CPU, Jetson Nano) per scan side
PAPER_F_RAW_HZ = {127: (83.2, 28.3), 255: (58.2, 22.3), 511: (21.0, 9.4)}
CPU_SECONDS = 10.0          # the CPU baseline keeps adding pairs until this much time has gone
PROFILE_STEPS = 50          # steps of the event-timed per-kernel pass (its event pool grows with them)


def source_digest() -> str:
    """sha256 over the library's HIP sources (names and contents, sorted)."""
    import hashlib
    src = os.path.join(ROOT, "paper_2203_00459_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(src)):
        if f.endswith((".hip", ".hpp")):
            h.update(f.encode())
            with open(os.path.join(src, f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed FETCH_SIZE/WRITE_SIZE
    summary (scaled by its copy-kernel calibration), or None when the summary is
    missing or was taken on other sources than the ones built here."""
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    meta = {}
    for ln in lines:
        if ln.startswith("# source-digest "):
            meta["digest"] = ln.split()[2]
        elif ln.startswith("# calibration-fetch "):
            meta["ff"] = float(ln.split()[2])
        elif ln.startswith("# calibration-write "):
            meta["fw"] = float(ln.split()[2])
    if meta.get("digest") != source_digest() or "ff" not in meta or "fw" not in meta:
        return None
    # rows: kernel, dispatches, fetch KiB, write KiB, MB; of a kernel's template
    # variants, the one with the most dispatches is the one the tuned plan ran
    best = None
    for ln in lines:
        if ln.startswith("#") or not ln.strip():
            continue
        parts = ln.split()
        name = ln[:34].strip().split("<")[0]
        if name == kernel and len(parts) >= 5:
            count, fetch, write = int(parts[-4]), float(parts[-3]), float(parts[-2])
            if best is None or count > best[0]:
                best = (count, fetch, write)
    if best is None:
        return None
    return (best[1] * meta["ff"] + best[2] * meta["fw"]) * 1024.0


def kernel_bytes(n: int, n_theta: int, n_r: int, batch: int, masked: bool, keep: bool = False) -> dict:
    """Algorithmic HBM bytes per launch of each kernel: compulsory reads of its
    inputs plus writes of its outputs, each touched once (float32 / complex64).
    keep: the training forward keeps its intermediates for the adjoint (k_rotate
    runs once and also writes d g'/d theta; k_rows1 / k_cols1 / k_rows2 run
    once).  Without keep the adjoint runs them again; kb_rows_fwd2 always
    transforms only the d c_xy lag rows."""
    N2 = n * n
    nrb = (n_r + max(2048 // n_theta, 4) - 1) // max(2048 // n_theta, 4)   # radius blocks of the polar pass
    hk = n_theta // 2 + 1
    m = 2 if masked else 1
    half = 2 * n * (n // 2) * 8            # both half spectra, complex64
    mag = 2 * n * (n // 2 + 1) * 4          # both magnitude half-planes, float32
    polar = 2 * n_r * n_theta * 4           # both polar adjoints, float32
    h2 = 3 * n // 4 + 1                     # unique columns of the 3n/2-point stage-2 rows
    rows2 = n * h2 * 16                     # stage-2 row spectra (F, G'), complex64 pairs
    lag = n * h2 * 8                        # stage-2 lag rows, complex64
    m2 = {127: 192, 255: 384, 511: 768}.get(n, 3 * n // 2)   # odd sides: stage-2 line length
    return {
        # forward
        "k_rows1": batch * (m * 2 * 4 * N2 + half),
        "k_cols1": batch * (half + mag),
        # with keep it also writes the per-radius angular spectra for the adjoint
        "k_polar": batch * (mag + nrb * hk * 8 + (n_r * n_theta * 8 if keep else 0)),
        "k_angle_fin": batch * (nrb * hk * 8 + n_theta * 4),
        # without keep k_rotate runs twice per step: forward (g') and adjoint (g', d g'/d theta)
        "k_rotate": batch * (m * 4 * N2 + (8 * N2 if keep else 6 * N2)),
        "k_rows2": batch * (m * 4 * N2 + 4 * N2 + rows2),
        "k_cols2": batch * (rows2 + lag),
        "k_rows3": batch * (lag + N2 * 4),
        "k_xy_fin": batch * 64,
        # adjoint (without keep, k_rows1, k_cols1 and k_rows2 run again to recompute their spectra)
        "kb_rows_fwd2": batch * (4 * N2 + lag),
        "kb_cols_xy": batch * (rows2 + lag + rows2),
        "kb_rows_xy": batch * (rows2 + 4 * N2 + 2 * N2 * 4),
        "kb_rotate_adj": batch * (4 * N2 + 4 * N2),
        "kb_dtheta": batch * (n_theta * 4 + n_theta * 8),
        "kb_polar": batch * (mag + polar),
        "kb_dmag": batch * (polar + mag),
        "kb_cols_mag": batch * (half + mag + half),
        "kb_rows_final": batch * (half + 2 * N2 * 4 + m * 2 * 4 * N2 + 2 * N2 * 4 + (m - 1) * 2 * N2 * 4),
        # odd sides (the paper's 127 / 255 / 511 px): stage-1 half spectra of (n + 1)/2
        # columns, stage 2 padded to m2 = 3 2^b with m2/2 + 1 columns
        "ko_rows1": batch * (m * 2 * 4 * N2 + n * ((n + 1) // 2) * 16),
        "ko_cols1": batch * (n * ((n + 1) // 2) * (16 + 8)),
        "ko_polar": batch * (n * ((n + 1) // 2) * 8),
        "ko_rotate": batch * (m * 4 * N2 + 4 * N2),
        "ko_rows2": batch * (m * 4 * N2 + 4 * N2 + n * (m2 // 2 + 1) * 16),
        "ko_cols2": batch * (n * (m2 // 2 + 1) * (16 + 8)),
        "ko_rows3": batch * (n * (m2 // 2 + 1) * 8 + 4 * N2),
    }


def pass_model_bytes(n: int) -> dict:
    """HBM bytes per pair of each kernel on the pass model of the method's
    steps (fp32 data, complex64 intermediates, ZeroPad to 2n, every
    pass reading its inputs and writing its outputs once).  These are the
    figures the roofline's `achieved` uses; the library's own per-launch model
    (``kernel_bytes``: 3n/2 padding, the passes as this library fuses them) is
    reported beside it.  Kernels that share one pass of the model get the
    pass's bytes once, on the kernel that moves them."""
    N2 = n * n
    return {
        "k_rows1": 16 * N2,        # S2 rows R2C
        "k_cols1": 12 * N2,        # S3 columns + |F|
        "k_polar": 4 * N2,         # S4 polar gather + angular FFT + sum over r
        "k_rows2": 24 * N2,        # S6 rotate + 2n rows (k_rotate is part of this pass)
        "k_cols2": 24 * N2,        # S7 columns fwd . conj . inv
        "k_rows3": 12 * N2,        # S8 inverse rows + softmax
        "kb_rows_fwd2": 40 * N2,   # translation adjoint: padded rows of f_w, g' and dc
        "kb_cols_xy": 40 * N2,     # column adjoint
        "kb_rows_xy": 28 * N2,     # inverse rows + dtheta_2
        "kb_rotate_adj": 8 * N2,   # Rotate transpose
        "kb_polar": 12 * N2,       # angular adjoint
        "kb_dmag": 12 * N2,        # CSR transpose gather
        "kb_cols_mag": 20 * N2,    # column adjoint with recomputed F
        "kb_rows_final": 24 * N2,  # final rows + Hann + mask
        # odd sides: the same passes
        "ko_rows1": 16 * N2, "ko_cols1": 12 * N2, "ko_polar": 4 * N2, "ko_rows2": 24 * N2,
        "ko_cols2": 24 * N2, "ko_rows3": 12 * N2,
    }


def cpu_description() -> str:
    """Model name, family/model/stepping and logical CPU count of the host (Linux)."""
    info = {}
    try:
        for ln in open("/proc/cpuinfo"):
            if ":" in ln:
                k, v = ln.split(":", 1)
                info.setdefault(k.strip(), v.strip())
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 0
    return (f"{info.get('model name', 'unknown')} (family {info.get('cpu family', '?')}, model "
            f"{info.get('model', '?')}, stepping {info.get('stepping', '?')}), {usable} usable of "
            f"{os.cpu_count()} logical CPUs")


def oracle_leg(run, n_items: int, threads: int, min_runs: int, seconds: float):
    """Time `run(i)` on the host with torch at `threads` threads: at least
    min_runs calls, then more until `seconds` have gone (at most four passes
    over the n_items inputs).  Returns (runs, seconds)."""
    import torch
    prev = torch.get_num_threads()
    torch.set_num_threads(threads)
    try:
        k = 0
        t0 = time.perf_counter()
        while k < 4 * n_items and (k < min_runs or time.perf_counter() - t0 < seconds):
            run(k % n_items)
            k += 1
        return k, time.perf_counter() - t0
    finally:
        torch.set_num_threads(prev)


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="batch512")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-pairs", type=int, default=4)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested): each scan pair is "
              "independent, so the batch would shard across GPUs with no exchange step; this "
              "build measures the one-GPU share.", file=sys.stderr)
        return 2
    from paper_2203_00459_amd import workloads
    if args.workload in workloads.RAGGED:
        return ragged_bench(args)
    if args.workload in workloads.TRAIN:
        return train_bench(args)
    if args.workload in workloads.TRAIN_RUN:
        return train_run_bench(args)
    if args.workload in workloads.INFER:
        return infer_bench(args)
    if args.workload in workloads.DRIVE:
        return drive_bench(args)
    return search_bench(args)


def mask_layers(levels: int, base: int, channels: int = 1):
    """(c_in, c_out, level) of the mask network's convolutions in order."""
    ch = [base << l for l in range(levels)]
    out = []
    for l in range(levels):
        out += [(channels if l == 0 else ch[l - 1], ch[l], l), (ch[l], ch[l], l)]
    for l in range(levels - 2, -1, -1):
        out += [(ch[l + 1] + ch[l], ch[l], l), (ch[l], ch[l], l)]
    return out


def mask_kernel_model(images: int, n: int, levels: int = 4, base: int = 8, channels: int = 1) -> dict:
    """Algorithmic HBM bytes and flops per training step of the mask network's
    kernel groups: every tensor read and written once (BF16 activations, FP32
    gradients), convolution flops 2 * pixels * 9 * c_in * c_out."""
    m = {}

    def add(k, b, f=0.0):
        bb, ff = m.get(k, (0.0, 0.0))
        m[k] = (bb + b, ff + f)

    for j, (ci, co, l) in enumerate(mask_layers(levels, base, channels)):
        px = images * (n >> l) ** 2
        cik = max(ci, 8)
        add("m_conv_fwd", px * (cik + co) * 2, 2.0 * px * 9 * ci * co)
        add("m_bn_relu", px * co * 4)
        add("m_bn_bwd", px * co * (4 + 2) * 2 + px * co * 2)
        add("m_wgrad", px * (co + cik) * 2, 2.0 * px * 9 * ci * co)
        if j:
            add("m_conv_dgrad", px * (co * 2 + ci * 4), 2.0 * px * 9 * ci * co)
    return m


def mask_infer_model(images: int, n: int, levels: int = 4, base: int = 8, channels: int = 1) -> dict:
    """Algorithmic HBM bytes and flops of the fused inference pass: every
    tensor it reads or writes once.  The first convolution reads the FP32
    scans, a decoder's first reads the skip activation and the deeper one at a
    quarter of its pixels, an encoder's second also writes the pooled output;
    the head reads the last activation and writes FP32 masks."""
    conv_b, flops = 0.0, 0.0
    layers = mask_layers(levels, base, channels)
    for j, (ci, co, l) in enumerate(layers):
        px = images * (n >> l) ** 2
        if j == 0:
            rd = px * channels * 4
        elif j >= 2 * levels and (j - 2 * levels) % 2 == 0:
            rd = px * (ci // 3) * 2 + px * (2 * ci // 3) * 2 / 4
        else:
            rd = px * ci * 2
        wr = px * co * 2 + (px * co * 2 / 4 if j < 2 * levels and j % 2 == 1 and l + 1 < levels else 0)
        conv_b += rd + wr
        flops += 2.0 * px * 9 * ci * co
    px0 = images * n * n
    return {"m_conv_fwd": (conv_b, flops), "m_head_fwd": (px0 * base * 2 + px0 * channels * 4, 0.0)}


def infer_bench(args) -> int:
    """One step = one inference pass of the mask network (running statistics)
    over both scans of every pair of the batch, as inside the masked ragged
    launch."""
    import numpy as np
    import torch

    from paper_2203_00459_amd import fmbym, synth, workloads
    from paper_2203_00459_amd.train import he_init

    cfg = workloads.INFER[args.workload]
    B, n, levels = cfg["pairs"], cfg["n"], cfg["levels"]
    f, g, _ = synth.make_batch(cfg["scenes"], B, split="bench")
    X = torch.from_numpy(np.concatenate([f, g])).to("cuda:0")
    params = he_init(levels, 8, 0)
    net = fmbym.MaskNet(params, levels=levels, base=8)
    # running statistics as a trained network has them (not the initial 0 / 1)
    nb = net.bn_running.numel() // 2
    rs = np.random.Generator(np.random.PCG64(7))
    net.bn_running.copy_(torch.from_numpy(np.concatenate([0.1 * rs.standard_normal(nb), 0.5 + rs.random(nb)])
                                          .astype(np.float32)).to("cuda:0"))
    for _ in range(args.warmup):
        net.forward(X, training=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        net.forward(X, training=False)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    psteps = min(args.steps, PROFILE_STEPS)
    fmbym.profile_enable(psteps * 64)
    for _ in range(psteps):
        net.forward(X, training=False)
    torch.cuda.synchronize()
    prof = fmbym.profile_read()
    fmbym.profile_enable(0)
    per_step = {k: t / psteps for k, (t, c) in prof.items()}
    mk = mask_infer_model(2 * B, n, levels)
    conv_ms = per_step.get("m_conv_fwd", 0.0)
    achieved = mk["m_conv_fwd"][0] / (conv_ms * 1e-3) / 1e9
    path_b = sum(b for b, _ in mk.values())
    res = {
        "metric": f"images/sec, {n}^2 mask-network inference ({levels} levels, running statistics), 1 GPU",
        "value": 2 * B / (ms * 1e-3),
        "unit": "images/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 conv (fp32 accumulate)", "data": "synthetic",
        "config": {"workload": args.workload, "images": 2 * B, "n": n, "levels": levels,
                   "mask_params": int(net.params.numel())},
        "roofline": {"bound": "hbm", "kernel": "m_conv_fwd (every convolution of the pass)", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "conv_fwd_mfma": {"achieved": mk["m_conv_fwd"][1] / (conv_ms * 1e-3) / 1e12, "peak": BF16_PEAK_TFLOPS,
                          "unit": "TFLOP/s", "frac": mk["m_conv_fwd"][1] / (conv_ms * 1e-3) / 1e12 / BF16_PEAK_TFLOPS},
        "roofline_path": {"bytes": path_b, "achieved": path_b / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                          "frac": path_b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernels_ms_per_step": {k: round(v, 5) for k, v in sorted(per_step.items())},
    }
    if not args.no_cpu_baseline:
        from oracle import mask_oracle as M
        th = torch.from_numpy(params).double()
        run_mean = net.bn_running[:nb].double().cpu()
        run_var = net.bn_running[nb:].double().cpu()
        done, t0 = 0, time.perf_counter()
        while done < 2 * B and (done < 1 or time.perf_counter() - t0 < CPU_SECONDS):
            x = X[done:done + 1].double().cpu()
            M.forward_eval(x, th, levels, 8, run_mean, run_var)
            done += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done / dt, "unit": "images/s", "cores": torch.get_num_threads(),
                               "cpu": cpu_description(), "kind": "oracle",
                               "sample": f"{done} images (about {CPU_SECONDS:.0f} s): FP64 oracle inference forward"}
    print(json.dumps(res), flush=True)
    return 0


def train_bench(args) -> int:
    """One step = one training step of the masked search (Eq. 10-13): mask
    network forward on both scans of every pair, masked search forward, pose
    loss, search adjoint, network adjoint, Adam."""
    import numpy as np
    import torch

    from paper_2203_00459_amd import fmbym, synth, workloads
    from paper_2203_00459_amd.train import MaskedSearchTrainer, TrainConfig

    cfg = workloads.TRAIN[args.workload]
    B, n, levels = cfg["batch"], cfg["n"], cfg["levels"]
    C = cfg.get("channels", 1)
    loss = fmbym.FMBYM_LOSS_L1 if cfg.get("loss") == "l1" else fmbym.FMBYM_LOSS_L2
    kw = workloads.search_kwargs(cfg["search"])
    dev = torch.device("cuda:0")
    pool = 4 * B
    f, g, p = synth.make_batch(cfg["scenes"], pool, split="bench")
    F, G, P = (torch.from_numpy(a).to(dev) for a in (f, g, p.astype(np.float32)))
    tr = MaskedSearchTrainer(kw, batch=B, cfg=TrainConfig(levels=levels, lr=1e-4, channels=C, loss=loss))
    batches = [(F[k * B:(k + 1) * B].contiguous(), G[k * B:(k + 1) * B].contiguous(),
                P[k * B:(k + 1) * B].contiguous()) for k in range(pool // B)]

    def step(i):
        tr.step(*batches[i % len(batches)])

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for i in range(args.steps):
        step(i)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    rf = train_roofline(step, min(args.steps, PROFILE_STEPS), B, n, kw, levels, C)
    res = {
        "metric": f"scan-pairs/sec, {n}^2 masked-search training step (mask net fwd+bwd, search fwd+bwd, Adam), 1 GPU",
        "value": B / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 conv (fp32 accumulate), f32 search", "data": "synthetic",
        "config": {"workload": args.workload, "batch": B, "n": n, "levels": levels, "channels": C,
                   "mask_params": int(tr.net.params.numel()), "loss": "l1" if loss == fmbym.FMBYM_LOSS_L1 else "l2",
                   "images_per_step": 2 * B},
        **rf,
    }
    if not args.no_cpu_baseline:
        from oracle import fmbym_oracle as O
        from oracle import mask_oracle as M
        from paper_2203_00459_amd.train import he_init
        th = torch.from_numpy(he_init(levels, 8, 0, C)).double().requires_grad_(True)
        done = 0
        t0 = time.perf_counter()
        while done < B and (done < 1 or time.perf_counter() - t0 < CPU_SECONDS):
            X = torch.from_numpy(np.stack([f[done], g[done]])).double()
            m = M.forward(X, th, levels, 8) if C == 1 else M.forward(X[None], th, levels, 8, ch=2)[0]
            pose = O.search(f[done], g[done], O.Params(**kw), m[0], m[1])["pose"]
            M.pose_loss(pose[None], torch.from_numpy(p[done:done + 1]).double(),
                        "l1" if loss == fmbym.FMBYM_LOSS_L1 else "l2").backward()
            done += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done / dt, "unit": "pairs/s", "cores": torch.get_num_threads(), "cpu": cpu_description(),
                               "kind": "oracle",
                               "sample": f"{done} pairs (about {CPU_SECONDS:.0f} s): FP64 oracle mask network + "
                                         f"masked search + {'L1' if loss == fmbym.FMBYM_LOSS_L1 else 'L2'} loss, "
                                         "autograd"}
    print(json.dumps(res), flush=True)
    return 0


def train_roofline(step, psteps: int, B: int, n: int, kw: dict, levels: int, C: int) -> dict:
    """Per-kernel event times over `psteps` training steps (step(i) runs step i):
    the dominant kernel against HBM on the network's byte model (or the search's),
    the forward convolutions against the BF16 matrix-core peak, and every kernel's
    time per step."""
    import torch

    from paper_2203_00459_amd import fmbym

    fmbym.profile_enable(psteps * 600)
    for i in range(psteps):
        step(i)
    torch.cuda.synchronize()
    prof = fmbym.profile_read()
    fmbym.profile_enable(0)
    per_step = {k: t / psteps for k, (t, c) in prof.items()}
    dom = max(per_step, key=per_step.get)
    mk = mask_kernel_model(2 * B // C, n, levels, 8, C)   # samples per network call
    sb = kernel_bytes(n, kw["n_theta"], n, B, masked=True, keep=True)
    byts = mk[dom][0] if dom in mk else sb.get(dom, 0)
    achieved = byts / (per_step[dom] * 1e-3) / 1e9
    conv_t = per_step.get("m_conv_fwd", 0.0) * 1e-3
    return {
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None},
        "conv_fwd_mfma": None if not conv_t else {
            "achieved": mk["m_conv_fwd"][1] / conv_t / 1e12, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": mk["m_conv_fwd"][1] / conv_t / 1e12 / BF16_PEAK_TFLOPS},
        "kernels_ms_per_step": {k: round(v, 5) for k, v in sorted(per_step.items())},
    }


def held_out_errors(tr, F, G, P) -> dict:
    """Errors of the masked search (network in inference mode) and of the
    unmasked search on held-out pairs: mean heading error (deg), mean and median
    translation error (m), and the fraction of pairs off by more than 20 degrees
    or 2 m."""
    import torch

    with torch.no_grad():
        m_f, m_g = tr.masks(F, G, training=False)
        pm = tr.search.forward(F, G, m_f, m_g, surfaces=False)["pose"]
        pu = tr.search.forward(F, G, surfaces=False)["pose"]

    def err(pose):
        d = (pose - P).double()
        th = d[:, 0].abs() * (180.0 / math.pi)
        t = d[:, 1:].norm(dim=1)
        return {"theta_deg": float(th.mean()), "t_m": float(t.mean()), "t_m_median": float(t.median()),
                "off_20deg_or_2m": float(((th > 20.0) | (t > 2.0)).double().mean())}

    return {"masked": err(pm), "unmasked": err(pu)}


def train_run_bench(args) -> int:
    """The configured mask-learning run: a generated training set trained for
    whole epochs (batch B, Adam), once per loss from the same initialisation and
    data order, each judged on held-out pairs against the unmasked search.  The
    headline rate is the first loss's training steps after `warmup` untimed
    ones (held-out evaluations between epochs are outside the timed segments)."""
    import numpy as np
    import torch

    from paper_2203_00459_amd import synth, workloads

    cfg = workloads.TRAIN_RUN[args.workload]
    B, n_pairs, n_test = cfg["batch"], cfg["pairs"], cfg["held_out"]
    t0 = time.perf_counter()
    f, g, p = synth.make_batch_parallel(cfg["scenes"], n_pairs, split="train")
    ft, gt, pt = synth.make_batch(cfg["scenes"], n_test, split="test")
    print(f"generated {n_pairs} training and {n_test} held-out pairs in {time.perf_counter() - t0:.0f} s",
          file=sys.stderr, flush=True)

    from paper_2203_00459_amd import fmbym
    from paper_2203_00459_amd.train import MaskedSearchTrainer, TrainConfig

    dev = torch.device("cuda:0")
    F, G, P = (torch.from_numpy(a).to(dev) for a in (f, g, p.astype(np.float32)))
    Ft, Gt, Pt = (torch.from_numpy(a).to(dev) for a in (ft, gt, pt.astype(np.float32)))
    del f, g
    kw = workloads.search_kwargs(cfg["search"])
    per_epoch = n_pairs // B
    losses_out, headline = {}, None
    for li, loss_name in enumerate(cfg["losses"]):
        loss = fmbym.FMBYM_LOSS_L1 if loss_name == "l1" else fmbym.FMBYM_LOSS_L2
        tr = MaskedSearchTrainer(kw, batch=n_test, cfg=TrainConfig(levels=cfg["levels"], lr=cfg["lr"], loss=loss))
        rng = np.random.Generator(np.random.PCG64(0))
        rec = {"before": held_out_errors(tr, Ft, Gt, Pt)}
        step_losses, timed_ms, timed_steps = [], 0.0, 0
        warm = min(args.warmup, per_epoch) if li == 0 else 0
        for epoch in range(cfg["epochs"]):
            perm = torch.from_numpy(rng.permutation(n_pairs)).to(dev)
            first = warm if epoch == 0 else 0
            for i in range(first):
                idx = perm[i * B:(i + 1) * B]
                step_losses.append(tr.step(F[idx].contiguous(), G[idx].contiguous(), P[idx].contiguous())[0])
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for i in range(first, per_epoch):
                idx = perm[i * B:(i + 1) * B]
                step_losses.append(tr.step(F[idx].contiguous(), G[idx].contiguous(), P[idx].contiguous())[0])
            ev1.record()
            torch.cuda.synchronize()
            timed_ms += ev0.elapsed_time(ev1)
            timed_steps += per_epoch - first
            rec[f"epoch{epoch + 1}"] = held_out_errors(tr, Ft, Gt, Pt)
            print(f"{loss_name} epoch {epoch + 1}: {rec[f'epoch{epoch + 1}']}", file=sys.stderr, flush=True)
        sl = torch.stack(step_losses).double().cpu().numpy().reshape(-1)
        rec["loss_first50"], rec["loss_last50"] = float(sl[:50].mean()), float(sl[-50:].mean())
        rec["ms_per_step"] = timed_ms / timed_steps
        rec["use_mask"] = bool(tr.evaluate(Ft, Gt, Pt)["use_mask"])
        losses_out[loss_name] = rec
        if li == 0:
            headline = (timed_ms, timed_steps, tr)

    timed_ms, timed_steps, tr = headline
    ms = timed_ms / timed_steps
    bi = [(F[k * B:(k + 1) * B].contiguous(), G[k * B:(k + 1) * B].contiguous(),
           P[k * B:(k + 1) * B].contiguous()) for k in range(4)]
    rf = train_roofline(lambda i: tr.step(*bi[i % 4]), PROFILE_STEPS, B, kw["n"], kw, cfg["levels"], 1)
    res = {
        "metric": f"scan-pairs/sec, {kw['n']}^2 masked-search training ({n_pairs} pairs, batch {B}, "
                  f"{cfg['losses'][0].upper()} pose loss), 1 GPU",
        "value": B / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": timed_steps, "warmup": min(args.warmup, per_epoch), "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16 conv (fp32 accumulate), f32 search", "data": "synthetic",
        "config": {"workload": args.workload, "pairs": n_pairs, "held_out": n_test, "batch": B,
                   "epochs": cfg["epochs"], "lr": cfg["lr"], "levels": cfg["levels"], "losses": list(cfg["losses"]),
                   "order": "PCG64(0) permutation per epoch, the same for every loss"},
        "gain": losses_out,
        **rf,
        "cpu_baseline": None,
    }
    print(json.dumps(res), flush=True)
    return 0


def drive_bench(args) -> int:
    """One step = the forward search over every consecutive pair of a drive in
    one launch (f = scans[:-1], g = scans[1:], overlapping views of one array);
    the poses are chained into a trajectory and scored over 100 ... 800 m
    segments against the drive's true poses."""
    import numpy as np
    import torch

    from paper_2203_00459_amd import fmbym, odometry, synth, workloads

    cfg = workloads.DRIVE[args.workload]
    kw = workloads.search_kwargs(cfg["search"])
    scans_np, gt, rel_true = synth.make_drive(cfg["drive"], split="bench")
    dev = torch.device("cuda:0")
    S = torch.from_numpy(scans_np).to(dev)
    P = len(scans_np) - 1
    n, nt = kw["n"], kw["n_theta"]
    s = fmbym.Search(max_batch=P, **kw)
    tuning, _ = fmbym.plan_autotune(s.plan, P, False, dev)
    f, g = S[:-1], S[1:]
    for _ in range(args.warmup):
        out = s.forward(f, g, surfaces=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        out = s.forward(f, g, surfaces=False)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    rel = out["pose"].double().cpu().numpy()
    drift = odometry.segment_errors(gt, odometry.chain(rel))
    gated, rejected = odometry.gate_outliers(rel)
    drift_gated = odometry.segment_errors(gt, odometry.chain(gated))
    # the same drive under the alternative readings of the scores (untimed)
    readings = {}
    for name, opt in (("hard_argmax", dict(hard_argmax=True)), ("logit_zscore", dict(zscore=True))):
        sr = fmbym.Search(max_batch=P, **kw, **opt)
        r = sr.forward(f, g, surfaces=False)["pose"].double().cpu().numpy()
        torch.cuda.synchronize()
        sr.close()
        e = odometry.segment_errors(gt, odometry.chain(r))
        t_err = np.hypot(*(r[:, 1:] - rel_true[:, 1:]).T)
        readings[name] = {"t_pct": e["t_pct"], "r_deg_per_km": e["r_deg_per_km"],
                          "pairs_t_err_over_1m": float((t_err > 1.0).mean())}
    pass_bytes = 92 * n * n * P
    res = {
        "metric": f"scan-pairs/sec, {n}^2 radar odometry (forward search over a drive's consecutive pairs), 1 GPU",
        "value": P / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "frames": len(scans_np), "pairs": P, "n": n, "n_theta": nt,
                   "pass": "fwd", "launch": "all pairs in one call"},
        "roofline_path": {"bound": "hbm", "bytes_per_step": pass_bytes,
                          "achieved": pass_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": pass_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "drift": {"t_pct": drift["t_pct"], "r_deg_per_km": drift["r_deg_per_km"],
                  "segments": drift["segments"],
                  "per_length_m": {str(k): {"t_pct": v[0], "r_deg_per_km": v[1], "segments": v[2]}
                                   for k, v in drift["per_length"].items()},
                  "drive_m": float(np.hypot(*np.diff(gt[:, :2], axis=0).T).sum())},
        # option beside the paper's chaining: pairs off the motion prior replaced
        "drift_gated": {"t_pct": drift_gated["t_pct"], "r_deg_per_km": drift_gated["r_deg_per_km"],
                        "segments": drift_gated["segments"], "rejected_pairs": int(rejected.sum())},
        "drift_readings": readings,
        "pairs_t_err_over_1m": float((np.hypot(*(rel[:, 1:] - rel_true[:, 1:]).T) > 1.0).mean()),
        "tuning": tuning,
    }
    if not args.no_cpu_baseline:
        from oracle import fmbym_oracle as O
        p = O.Params(**kw)
        t0 = time.perf_counter()
        done = 0
        while done < P and (done < 2 or time.perf_counter() - t0 < CPU_SECONDS):
            O.search(scans_np[done], scans_np[done + 1], p)
            done += 1
        dt = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": done / dt, "unit": "pairs/s", "cores": torch.get_num_threads(), "cpu": cpu_description(),
                               "kind": "oracle",
                               "sample": f"the drive's first {done} pairs (about 10 s), FP64 oracle forward"}
    print(json.dumps(res), flush=True)
    s.close()
    return 0


def ragged_bench(args) -> int:
    """One step = one captured launch of a ragged work list (forward search of
    every pair at its own size); reports pairs/s and per-pair latency."""
    import numpy as np
    import torch

    from paper_2203_00459_amd import fmbym, synth, workloads

    cfg = workloads.RAGGED[args.workload]
    names = synth.ragged_mix(cfg["n_pairs"], cfg["mix"])
    sizes = [name for name, _ in cfg["mix"]]
    dev = torch.device("cuda:0")
    counts = {k: names.count(k) for k in sizes}
    scans = {}
    for k in sizes:
        f, g, _ = synth.make_batch(k, counts[k], split="bench")
        scans[k] = (torch.from_numpy(f).to(dev), torch.from_numpy(g).to(dev))
    seen = {k: 0 for k in sizes}
    pairs = []
    masked = cfg.get("mask") == "net"
    for k in names:
        j = seen[k]
        seen[k] += 1
        pairs.append((scans[k][0][j], scans[k][1][j]) + (("net",) if masked else ()))
    searches = [fmbym.Search(max_batch=counts[k], **workloads.search_kwargs(k)) for k in sizes]
    net = None
    if masked:
        from paper_2203_00459_amd.train import he_init
        net = fmbym.MaskNet(he_init(4, 8, 0), levels=4)
    r = fmbym.Ragged(searches, pairs, net=net)
    for _ in range(args.warmup):
        r.launch()
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        r.launch()
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / args.steps
    lat = r.latencies_us().numpy()
    fwd = ("k_rows1", "k_cols1", "k_polar", "k_angle_fin", "k_rows2", "k_cols2", "k_rows3", "k_xy_fin",
           "k_rotate")
    nbytes = 0
    for k in sizes:
        kw = workloads.search_kwargs(k)
        kb = kernel_bytes(kw["n"], kw["n_theta"], kw["n"], counts[k], masked=False)
        nbytes += sum(kb[x] for x in fwd)
    achieved = nbytes / (ms * 1e-3) / 1e9
    res = {
        "metric": f"scan-pairs/sec, ragged {cfg['n_pairs']}-pair forward search (mixed sizes"
                  f"{', mask network inside the launch' if masked else ''}), 1 GPU",
        "value": cfg["n_pairs"] / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "pairs": counts, "pass": "fwd",
                   "masks": "4-level network, inference" if masked else "none",
                   "launch": "one captured graph per work list"},
        "latency_us": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "max": float(lat.max())},
        "roofline": {"bound": "hbm", "kernel": "whole launch (search forward bytes only)" if masked
                     else "whole launch", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        from oracle import fmbym_oracle as O
        # rounds of one pair of each size until about CPU_SECONDS of work; per-size
        # mean times weighted by the mix
        spent = {k: 0.0 for k in sizes}
        rounds = 0
        t_all = time.perf_counter()
        while rounds < min(counts.values()) and (rounds < 1 or time.perf_counter() - t_all < CPU_SECONDS):
            for k in sizes:
                p = O.Params(**workloads.search_kwargs(k))
                f, g = scans[k][0][rounds].cpu().numpy(), scans[k][1][rounds].cpu().numpy()
                t0 = time.perf_counter()
                O.search(f, g, p)
                spent[k] += time.perf_counter() - t0
            rounds += 1
        mean_t = sum(counts[k] * spent[k] / rounds for k in sizes) / cfg["n_pairs"]
        res["cpu_baseline"] = {"value": 1.0 / mean_t, "unit": "pairs/s", "cores": torch.get_num_threads(), "cpu": cpu_description(),
                               "kind": "oracle",
                               "sample": f"{rounds} pair(s) of each size (about {CPU_SECONDS:.0f} s), FP64 oracle "
                                         "forward, weighted by the mix"}
    print(json.dumps(res), flush=True)
    r.close()
    return 0


def search_bench(args) -> int:
    import numpy as np
    import torch

    from paper_2203_00459_amd import fmbym, synth, workloads

    cfg = workloads.SEARCH[args.workload]
    kw = workloads.search_kwargs(args.workload)
    B, n, nt = cfg["batch"], cfg["n"], cfg["n_theta"]
    dev = torch.device("cuda:0")
    mode = workloads.PASS.get(args.workload, "fwd+bwd")
    f_np, g_np, gt_pose = synth.make_batch(args.workload, B, split="bench")
    f = torch.from_numpy(f_np).to(dev)
    g = torch.from_numpy(g_np).to(dev)
    s = fmbym.Search(max_batch=B, **kw)
    with_bwd = mode == "fwd+bwd"
    out = s.forward(f, g)
    if with_bwd:
        try:
            s.backward(f, g, None, None, out, torch.ones(B, 3, device=dev))
        except fmbym.FmbymError as e:
            if e.code != fmbym.FMBYM_EUNSUPPORTED:
                raise
            with_bwd = False
    d_pose = torch.ones(B, 3, device=dev)
    # column-tile widths measured on this GPU for this workload (untimed; results do not depend on them)
    if n % 2:   # odd sides: no tunable column tiles (their column passes have fixed widths)
        tuning = fmbym.plan_get_tuning(s.plan)
    else:
        tuning, _ = fmbym.plan_autotune(s.plan, B, with_bwd, dev)
    torch.cuda.synchronize()

    if args.copy_probe_mb:
        src = torch.empty(args.copy_probe_mb << 18, device=dev)        # MiB of float32
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)   # a plain read+write kernel of known size
        torch.cuda.synchronize()
        del src, dst

    def step(keep=with_bwd, fused=True):
        # the training forward keeps its intermediates and the adjoint reads them;
        # fused: both in one fmbym_search_vjp call (each half of the batch runs
        # both passes on its stream, one fork and join), else the two calls
        if with_bwd and keep and fused:
            s.vjp(f, g, None, None, d_pose)
            return
        o = s.forward(f, g, keep=keep)
        if with_bwd:
            s.backward(f, g, None, None, o, d_pose)

    def timed(keep):
        for _ in range(args.warmup):
            step(keep)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(args.steps):
            step(keep)
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps

    ms = timed(with_bwd)
    # per-step times from events between the steps, in a pass of its own (the
    # mean above has no events inside its timed region)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    evs[0].record()
    for i in range(args.steps):
        step(with_bwd)
        evs[i + 1].record()
    torch.cuda.synchronize()
    per_step = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(args.steps))
    ms_median = per_step[len(per_step) // 2]
    # the adjoint that recomputes the spectra (fmbym_search + fmbym_search_backward), same step
    ms_recompute = timed(False) if with_bwd else None
    extra = {"ms_per_step_median": ms_median, "ms_per_step_p90": per_step[(9 * len(per_step)) // 10]}
    if with_bwd:
        # the same step as the two calls fmbym_search_train + fmbym_search_backward_state
        # (two forks and joins per step)
        for _ in range(args.warmup):
            step(True, fused=False)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            step(True, fused=False)
        e1.record()
        torch.cuda.synchronize()
        ms_pair = e0.elapsed_time(e1) / args.steps
        extra["training_pair_path"] = {"ms_per_step": ms_pair, "value": B / (ms_pair * 1e-3), "unit": "pairs/s",
                                       "calls": "fmbym_search_train, fmbym_search_backward_state"}
    if n % 2:
        # the paper's own timing is one pair per call (Table III(a)): the eager
        # forward at batch 1 on its own plan, beside its ThinkPad / Jetson figures
        s1 = fmbym.Search(max_batch=1, **kw)
        f1, g1 = f[:1].contiguous(), g[:1].contiguous()
        for _ in range(args.warmup):
            s1.forward(f1, g1, surfaces=False)
        torch.cuda.synchronize()
        iters = max(args.steps, 200)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            s1.forward(f1, g1, surfaces=False)
        e1.record()
        torch.cuda.synchronize()
        lat = e0.elapsed_time(e1) / iters
        s1.close()
        paper = PAPER_F_RAW_HZ.get(n)
        extra["batch1"] = {"ms_per_pair": lat, "hz": 1e3 / lat, "calls": "eager fmbym_search, one pair"}
        if paper:
            extra["paper_context"] = {"f_raw_hz": {"thinkpad_i7_cpu": paper[0], "jetson_nano": paper[1]},
                                      "note": "Table III(a): batch 1 on the paper's hardware; context, "
                                              "not a target"}
    if mode == "fwd" and B == 1:
        # one pair: a captured launch (one HIP graph replay per pair)
        r = fmbym.Ragged([s], [(f[0], g[0])], stamps=False)
        for _ in range(max(args.warmup, 50)):
            r.launch()
        torch.cuda.synchronize()
        iters = max(args.steps, 2000)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(iters):
            r.launch()
        e1.record()
        torch.cuda.synchronize()
        extra["eager_ms_per_pair"] = ms
        ms = e0.elapsed_time(e1) / iters
        extra["latency_us"] = ms * 1e3
        r.close()
    if mode.startswith("fwd+joint"):
        K = workloads.JOINT_ANGLES
        jo = s.joint(f, g, K)
        for _ in range(2):
            jo = s.joint(f, g, K)
        torch.cuda.synchronize()
        jsteps = max(3, args.steps // 10)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(jsteps):
            jo = s.joint(f, g, K)
        e1.record()
        torch.cuda.synchronize()
        ms_j = e0.elapsed_time(e1) / jsteps
        dec = s.forward(f, g, surfaces=False)["pose"].double().cpu().numpy()
        jp = jo["pose"].double().cpu().numpy()

        def errs(pz):
            return (float(np.median(np.abs(pz[:, 0] - gt_pose[:, 0]))),
                    float(np.median(np.hypot(pz[:, 1] - gt_pose[:, 1], pz[:, 2] - gt_pose[:, 2]))))
        (td, xd), (tj, xj) = errs(dec), errs(jp)
        extra["joint_comparator"] = {
            "n_angles": K, "ms_per_step": ms_j, "value": B / (ms_j * 1e-3), "unit": "pairs/s",
            "decoupled_speedup": ms_j / ms,
            "median_theta_err_rad": {"decoupled": td, "joint": tj},
            "median_t_err_m": {"decoupled": xd, "joint": xj}}

        # full-circle heading (stage 2 again at theta + pi) on the same scenes
        # with headings drawn over the whole circle
        fc_f, fc_g, fc_gt = synth.make_batch(args.workload, B, split="bench", theta_max_deg=180.0)
        Ff, Fg = torch.from_numpy(fc_f).to(dev), torch.from_numpy(fc_g).to(dev)
        for _ in range(args.warmup):
            fc = s.full_circle(Ff, Fg)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            fc = s.full_circle(Ff, Fg)
        e1.record()
        torch.cuda.synchronize()
        ms_fc = e0.elapsed_time(e1) / args.steps
        plain = s.forward(Ff, Fg, surfaces=False)["pose"].double().cpu().numpy()
        fcp = fc["pose"].double().cpu().numpy()

        def wrap(a):
            return (a + math.pi) % (2 * math.pi) - math.pi
        step_rad = math.pi / nt
        e_plain = np.abs(wrap(plain[:, 0] - fc_gt[:, 0]))
        e_fc = np.abs(wrap(fcp[:, 0] - fc_gt[:, 0]))
        # pass model: the forward (92 n^2) plus stage 2 again (S6-S8: 60 n^2)
        fc_bytes = (92 + 60) * n * n * B
        extra["full_circle"] = {
            "ms_per_step": ms_fc, "value": B / (ms_fc * 1e-3), "unit": "pairs/s",
            "vs_decoupled_forward": ms_fc / ms,
            "roofline_path": {"bound": "hbm", "bytes_per_step": fc_bytes,
                              "achieved": fc_bytes / (ms_fc * 1e-3) / 1e9, "peak": HBM_PEAK_GBS,
                              "unit": "GB/s", "frac": fc_bytes / (ms_fc * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "headings": "uniform over [-pi, pi)",
            "theta_within_2_bins": {"decoupled": float((e_plain <= 2 * step_rad).mean()),
                                    "full_circle": float((e_fc <= 2 * step_rad).mean())},
            "median_t_err_m": float(np.median(np.hypot(fcp[:, 1] - fc_gt[:, 1], fcp[:, 2] - fc_gt[:, 2])))}

    # second timed pass: HIP events around every library launch, on its stream;
    # the batch unsplit, so that every launch is one kernel over the whole batch
    # with nothing running beside it
    fmbym.plan_set_tuning(s.plan, dict(tuning, split=1))
    for _ in range(2):
        step()
    fmbym.profile_enable(min(args.steps, PROFILE_STEPS) * 96)
    for _ in range(min(args.steps, PROFILE_STEPS)):
        step()
    torch.cuda.synchronize()
    prof = fmbym.profile_read()
    fmbym.profile_enable(0)
    fmbym.plan_set_tuning(s.plan, tuning)
    per_kernel = {k: (t / c) for k, (t, c) in prof.items()}
    dom = max(prof, key=lambda k: prof[k][0])
    kb = kernel_bytes(n, nt, n, B, masked=False, keep=with_bwd)
    pm = pass_model_bytes(n)
    launch_s = per_kernel[dom] * 1e-3
    achieved = pm[dom] * B / launch_s / 1e9 if dom in pm else None
    achieved_lib = kb[dom] / launch_s / 1e9 if dom in kb else None

    if with_bwd:
        metric = "scan-pairs/sec, 512^2 decoupled search fwd+bwd, 1 GPU"
    elif mode == "fwd" and B == 1:
        metric = f"scan-pairs/sec, {n}^2 decoupled search forward, one pair per captured launch, 1 GPU"
    elif mode.startswith("fwd+joint"):
        metric = (f"scan-pairs/sec, {n}^2 decoupled search forward (beside the "
                  f"{workloads.JOINT_ANGLES}-heading joint comparator), 1 GPU")
    else:
        metric = f"scan-pairs/sec, {n}^2 decoupled search forward, 1 GPU"
    res = {
        "metric": metric,
        "value": B / (ms * 1e-3),
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "batch": B, "n": n, "n_theta": nt,
                   "pass": "fwd+bwd, one fmbym_search_vjp call per step (the forward keeps its "
                           "intermediates for the adjoint)" if with_bwd else mode},
        "roofline": {"bound": "hbm", "kernel": dom, "launch": "whole batch, unsplit (per-kernel pass)",
                     "launch_ms": per_kernel[dom],
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": None if achieved is None else achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(dom) if args.workload == "batch512" else None,
                     "algorithmic_bytes": None if dom not in pm else pm[dom] * B,
                     "byte_model": f"pass model, {pm[dom] // (n * n) if dom in pm else '?'} n^2 per pair",
                     "library_model": {"algorithmic_bytes": kb.get(dom), "achieved": achieved_lib,
                                       "frac": None if achieved_lib is None else achieved_lib / HBM_PEAK_GBS,
                                       "note": "the library's own passes: 3n/2 padding, fused stages"}},
        "kernels_ms": {k: round(v, 5) for k, v in sorted(per_kernel.items())},
    }
    # whole path against the pass model's bytes per pair (304 n^2 fwd+bwd, 92 n^2 fwd)
    pass_bytes = (304 if with_bwd else 92) * n * n * B
    res["roofline_path"] = {"bound": "hbm", "bytes_per_step": pass_bytes,
                            "achieved": pass_bytes / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": pass_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    res.update(extra)
    res["tuning"] = tuning
    if ms_recompute is not None:
        frac_rc = pass_bytes / (ms_recompute * 1e-3) / 1e9 / HBM_PEAK_GBS
        res["recompute_path"] = {"ms_per_step": ms_recompute, "value": B / (ms_recompute * 1e-3),
                                 "unit": "pairs/s", "frac": frac_rc, "target_frac": 0.5,
                                 "meets_target": frac_rc >= 0.5,
                                 "calls": "fmbym_search, fmbym_search_backward (spectra recomputed)"}

    from oracle import fmbym_oracle as O
    p = O.Params(**kw)
    # pose error against the FP64 oracle on sampled pairs of the timed batch
    # (the GPU poses of one more step on the same inputs)
    gpu_pose = (s.vjp(f, g, None, None, d_pose) if with_bwd else s.forward(f, g, surfaces=False))["pose"]
    gpu_pose = gpu_pose.double().cpu().numpy()
    sample = sorted({0, B // 3, (2 * B) // 3, B - 1})
    dth, dt_px = [], []
    for b in sample:
        ref = O.search(f_np[b], g_np[b], p)["pose"].numpy()
        dth.append(abs(gpu_pose[b, 0] - ref[0]))
        dt_px.append(float(np.hypot(gpu_pose[b, 1] - ref[1], gpu_pose[b, 2] - ref[2])) / kw["delta_xy"])
    res["pose_err_vs_oracle"] = {"pairs": sample, "max_theta_rad": float(max(dth)),
                                 "max_t_px": float(max(dt_px)), "max_t_m": float(max(dt_px)) * kw["delta_xy"],
                                 "bar": {"theta_rad": 1e-3, "t_px": 1e-3},
                                 "within_bar": bool(max(dth) <= 1e-3 and max(dt_px) <= 1e-3)}

    if not args.no_cpu_baseline:
        def run(b):
            if with_bwd:
                O.search_grad(f_np[b], g_np[b], [1.0, 1.0, 1.0], p)
            else:
                O.search(f_np[b], g_np[b], p)

        what = "forward + autograd backward" if with_bwd else "forward"
        threads = torch.get_num_threads()
        k, dt = oracle_leg(run, B, threads, args.cpu_pairs, CPU_SECONDS)
        k1, dt1 = oracle_leg(run, B, 1, 2, CPU_SECONDS)
        res["cpu_baseline"] = {"value": k / dt, "unit": "pairs/s", "cores": threads, "cpu": cpu_description(),
                               "kind": "oracle",
                               "sample": f"{k} oracle runs over {min(k, B)} of the {B} pairs, FP64 oracle {what}",
                               "one_thread": {"value": k1 / dt1, "unit": "pairs/s", "cores": 1,
                                              "sample": f"{k1} oracle runs over {min(k1, B)} of the {B} pairs"}}
    print(json.dumps(res), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
