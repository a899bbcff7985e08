"""Host-side parts of bench.py: the committed counter summary is parsed, and
its traffic figure is reported only while the kernel source is unchanged."""
import hashlib
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_traffic_is_read_from_the_committed_summary():
    if not os.path.exists(bench.PROFILE_SUMMARY):
        assert bench.measured_traffic() is None
        return
    text = open(bench.PROFILE_SUMMARY).read()
    src = bench.kernel_source_hash()
    t = bench.measured_traffic()
    if f"`{src}`" in text:
        assert t is not None and t > 0
    else:
        assert t is None


def test_traffic_is_dropped_when_the_source_changes(tmp_path, monkeypatch):
    summary = tmp_path / "summary.md"
    summary.write_text("traffic_bytes_per_launch: `123`\n\nkernel_source_sha256: `deadbeef` (of the kernel)\n")
    src = tmp_path / "kernel.h"
    src.write_bytes(b"// kernel\n")
    monkeypatch.setattr(bench, "PROFILE_SUMMARY", str(summary))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", [str(src)])
    assert bench.measured_traffic() is None
    good = hashlib.sha256(b"// kernel\n").hexdigest()
    summary.write_text(f"traffic_bytes_per_launch: `123`\n\nkernel_source_sha256: `{good}` (of the kernel)\n")
    assert bench.measured_traffic() == 123.0


def test_training_rate_uses_the_adam_step_time():
    hist = {"steps": 10, "batch": 4096, "step_seconds": 2.0}
    r = bench.training_rate(hist)
    assert r["flops"] == 10 * 4096 * bench.TRAIN_FLOPS_PER_SAMPLE
    assert abs(r["achieved"] - r["flops"] / 2.0 / 1e12) < 1e-9 and r["unit"] == "TFLOP/s"
    # forward 45*128 + 2*128*128 + 128*4 multiply-adds; backward adds the input
    # gradients of the three upper layers
    assert bench.MLP_FWD_MACS == 39040 and bench.MLP_BWD_MACS == 39040 + 33280


def test_valu_op_count_and_peak():
    """12 per candidate test, 70 per contact, 210 per floe-step otherwise;
    peak 256 CUs x 64 lanes x 2.4 GHz."""
    assert bench.valu_ops_per_floe_step(0, 0) == 210.0
    assert bench.valu_ops_per_floe_step(10, 0.5) == 120 + 35 + 210
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-9
