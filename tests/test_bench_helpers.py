"""Host-side parts of bench.py: the HBM-traffic lookup in the committed
counter summary and the refusal of more than one GPU (CPU only)."""
import bench


def test_traffic_lookup_scales_the_counted_kib_of_the_most_run_variant(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text(
        "# header\n"
        f"# source-digest {bench.source_digest()}  (sha256)\n"
        "# calibration-fetch 2.0\n"
        "# calibration-write 1.0\n"
        "\n"
        f"{'kernel':<34} {'dispatches':>10} {'fetch_KiB':>12} {'write_KiB':>12} {'hbm_MB':>10}\n"
        f"{'kb_cols_xy<512, 16>':<34} {26:>10d} {100.0:>12.1f} {50.0:>12.1f} {0.26:>10.2f}\n"
        f"{'kb_cols_xy<512, 4>':<34} {192:>10d} {10.0:>12.1f} {5.0:>12.1f} {0.03:>10.2f}\n"
        f"{'kb_dmag':<34} {244:>10d} {7.0:>12.1f} {3.0:>12.1f} {0.02:>10.2f}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("kb_cols_xy") == (10.0 * 2.0 + 5.0) * 1024.0
    assert bench.measured_traffic("kb_dmag") == (7.0 * 2.0 + 3.0) * 1024.0
    assert bench.measured_traffic("k_rows1") is None


def test_traffic_lookup_refuses_a_summary_of_other_sources(tmp_path, monkeypatch):
    f = tmp_path / "traffic.txt"
    f.write_text("# source-digest 0000000000000000\n# calibration-fetch 2.0\n# calibration-write 1.0\n"
                 f"{'kb_dmag':<34} {244:>10d} {7.0:>12.1f} {3.0:>12.1f} {0.02:>10.2f}\n")
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("kb_dmag") is None


def test_more_than_one_gpu_is_refused_before_any_device_work():
    """--gpus N > 1 exits with status 2 and says why, before importing the
    library or touching a device (runs on the CPU)."""
    import os
    import subprocess
    import sys
    here = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(here, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=here)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_inference_byte_model_counts_each_fused_tensor_once():
    """Two levels, one 32 x 32 image, counted by hand: the first convolution
    reads the FP32 scan, the encoder's second also writes the pooled level-1
    input, the decoder's first reads the skip activation and the deeper one
    at its own (quarter) size; the head reads the last activation and writes
    the FP32 mask."""
    import bench

    m = bench.mask_infer_model(1, 32, levels=2, base=8)
    p0, p1 = 32 * 32, 16 * 16
    conv = ((p0 * 4 + p0 * 16) + (p0 * 16 + p0 * 16 + p1 * 16) + (p1 * 16 + p1 * 32) + (p1 * 32 + p1 * 32)
            + (p0 * 16 + p1 * 32 + p0 * 16) + (p0 * 16 + p0 * 16))
    flops = 2 * 9 * (p0 * 1 * 8 + p0 * 8 * 8 + p1 * 8 * 16 + p1 * 16 * 16 + p0 * 24 * 8 + p0 * 8 * 8)
    assert m["m_conv_fwd"] == (conv, flops)
    assert m["m_head_fwd"] == (p0 * 16 + p0 * 4, 0.0)
