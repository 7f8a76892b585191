"""Host logic of bench.py (no GPU): algorithmic bytes, the source-hash
guard on committed counter values, and the ALU roofline arithmetic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_per_quad():
    # state in and out 2 x 108, parameters 24, action 16, goal 12, and the
    # observation row of 18 + 6 K floats
    assert bench.algorithmic_bytes_per_quad(6, 1) == 484
    assert bench.algorithmic_bytes_per_quad(0, 1) == 340
    assert bench.algorithmic_bytes_per_quad(6, 1, with_obs=False) == 256


def test_source_hash_covers_every_kernel_header(tmp_path, monkeypatch):
    csrc = tmp_path / "paper_2306_09537_amd" / "csrc"
    csrc.mkdir(parents=True)
    for f in bench.KERNEL_SOURCES:
        (tmp_path / f).write_bytes(b"x")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    names = {os.path.basename(f) for f in bench.KERNEL_SOURCES}
    assert names == {"qs_device.h", "qs_kernels.h", "qs_rollout.h", "qs_adjoint.h"}
    for f in bench.KERNEL_SOURCES:
        (tmp_path / f).write_bytes(b"y")
        assert bench.kernel_source_hash() != h0, f
        (tmp_path / f).write_bytes(b"x")
    assert bench.kernel_source_hash() == h0


def write_profile(tmp_path, monkeypatch, text):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / "p.md").write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


def test_counter_values_only_while_sources_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    write_profile(tmp_path, monkeypatch, "hash `abcdef0123456789`\n\nk_valu: 12\n")
    assert bench.measured_counter("p.md", "k_valu") == 12
    assert bench.measured_counter("p.md", "missing") is None
    assert bench.measured_counter("absent.md", "k_valu") is None
    write_profile(tmp_path, monkeypatch, "hash `ffffffffffffffff`\n\nk_valu: 12\n")
    assert bench.measured_counter("p.md", "k_valu") is None


def test_alu_roofline_arithmetic(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    # 1 ms at 2457.6 G SIMD-cycles/s is 2,457,600,000 available cycles
    write_profile(tmp_path, monkeypatch, "`abcdef0123456789`\n"
                  "x_valu_busy_lo_cycles: 1228800000\n"
                  "x_valu_busy_hi_cycles: 1843200000\n"
                  "x_fp32_flops: 15730000000\n")
    r = bench.alu_roofline("p.md", "x_", 1.0)
    assert r["bound"] == "alu"
    assert r["peak"] == pytest.approx(2457.6)
    assert r["frac"] == pytest.approx(0.5)
    assert r["frac_upper"] == pytest.approx(0.75)
    assert r["achieved"] == pytest.approx(1228.8)
    assert r["fp32_tflops"] == pytest.approx(15.73)
    assert r["fp32_frac_of_157_3"] == pytest.approx(0.1)
    assert bench.alu_roofline("p.md", "y_", 1.0) is None


def test_fwdbwd_alu_needs_matching_horizon(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    write_profile(tmp_path, monkeypatch, "`abcdef0123456789`\n"
                  "fwdbwd_horizon: 200\n"
                  "backward_valu_busy_lo_cycles: 2457600\n"
                  "backward_valu_busy_hi_cycles: 2457600\n"
                  "backward_fp32_flops: 1\n")
    monkeypatch.setattr(bench, "FWDBWD_PROFILES", {"w": ("p.md", "")})
    assert bench.fwdbwd_alu("w", 200, "backward_", 1.0)["frac"] == pytest.approx(1e-3)
    assert bench.fwdbwd_alu("w", 100, "backward_", 1.0) is None
    assert bench.fwdbwd_alu("other", 200, "backward_", 1.0) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_fwdbwd_counter_needs_matching_horizon(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    write_profile(tmp_path, monkeypatch, "`abcdef0123456789`\n"
                  "fwdbwd_horizon: 200\n"
                  "backward_traffic_bytes: 496901258\n")
    monkeypatch.setattr(bench, "FWDBWD_PROFILES", {"w": ("p.md", "")})
    assert bench.fwdbwd_counter("w", 200, "backward_traffic_bytes") == 496901258
    assert bench.fwdbwd_counter("w", 100, "backward_traffic_bytes") is None
    assert bench.fwdbwd_counter("other", 200, "backward_traffic_bytes") is None


def test_launch_traffic_per_workload():
    # the committed summaries carry the counter bytes of every timed
    # one-substep workload, on the current kernel sources
    for wl in ("swarm8", "scale32", "scale1"):
        t = bench.launch_traffic(wl, 1)
        assert t is None or t > 0
    assert bench.launch_traffic("swarm8", 10) is None
    assert bench.launch_traffic("uneven", 1) is None
