"""Host logic of bench.py (no GPU): algorithmic bytes and operations, the
source-hash guard on committed counter values, and the roofline
arithmetic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_2306_09537_amd import workloads as W  # noqa: E402


def test_algorithmic_bytes_per_quad():
    # state in and out 2 x 108, parameters 24, action 16, goal 12, and the
    # observation row of 18 + 6 K floats
    assert bench.algorithmic_bytes_per_quad(6, 1) == 484
    assert bench.algorithmic_bytes_per_quad(0, 1) == 340
    assert bench.algorithmic_bytes_per_quad(6, 10) == 484
    assert bench.algorithmic_bytes_per_quad(6, 1, with_obs=False) == 256


def test_backward_bytes():
    # 1024 x 8 quads, 200 substeps, checkpoints every 20: the tape written
    # and read, actions twice, action gradient; per segment checkpoint and
    # parameters; once adjoint in/out, parameters and their gradient
    Q = 8192
    assert bench.backward_bytes(Q, 200, 1, 20) == Q * (200 * 296 + 10 * 132 + 296)


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


def write_profile(tmp_path, monkeypatch, text, name="p.md"):
    (tmp_path / "profiles").mkdir(exist_ok=True)
    (tmp_path / "profiles" / name).write_text(text)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))


def test_counter_values_only_while_sources_match(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    write_profile(tmp_path, monkeypatch, "hash `abcdef0123456789`\n\nk_valu: 12\n  f: 1.5\n")
    assert bench.profile_value("p.md", "k_valu") == 12
    assert bench.profile_value("p.md", "f") == 1.5
    assert bench.profile_value("p.md", "missing") is None
    assert bench.profile_value("absent.md", "k_valu") is None
    write_profile(tmp_path, monkeypatch, "hash `ffffffffffffffff`\n\nk_valu: 12\n")
    assert bench.profile_value("p.md", "k_valu") is None
    assert bench.profile_value("p.md", "k_valu", need_hash=False) == 12


def test_alu_roofline_arithmetic(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "abcdef0123456789")
    # 15.73 G operations in 1 ms: 15.73 TFLOP/s, a tenth of the FP32 peak;
    # 614,400,000 issued VALU instructions x 4 cycles fill half of the
    # 2,457,600,000 SIMD-cycles of 1 ms
    write_profile(tmp_path, monkeypatch, "`abcdef0123456789`\n"
                  "x_valu_insts: 491520000\n"
                  "x_fp32_valu_insts: 245760000\n"
                  "x_active_inst_valu: 307200000\n")
    r = bench.alu_roofline(15.73e9, 1.0, "p.md", "x_")
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["peak"] == pytest.approx(157.3)
    assert r["achieved"] == pytest.approx(15.73)
    assert r["frac"] == pytest.approx(0.1)
    assert r["valu_lane_ops_per_alg_flop"] == pytest.approx(491520000 * 64 / 15.73e9)
    assert r["fp32_lane_ops_per_alg_flop"] == pytest.approx(245760000 * 64 / 15.73e9)
    assert r["valu_issue_util"] == pytest.approx(0.5)
    assert bench.alu_roofline(None, 1.0) is None
    bare = bench.alu_roofline(15.73e9, 1.0, "p.md", "y_")
    assert "valu_issue_util" not in bare and bare["frac"] == pytest.approx(0.1)


def test_hbm_roofline_arithmetic():
    r = bench.hbm_roofline(8_000_000, 0.002, traffic=4_000_000)
    assert r["achieved"] == pytest.approx(4000.0)
    assert r["frac"] == pytest.approx(0.5)
    assert r["traffic_frac"] == pytest.approx(0.25)
    assert bench.hbm_roofline(8_000_000, 0.002)["traffic_frac"] is None


def test_call_flops_from_the_committed_counts():
    # the op-counting oracle's table is committed for every workload
    for mk in (W.swarm8, W.scale32, W.scale1, W.uneven, W.diff, W.plain):
        w = mk(seed=0) if mk is not W.scale1 else mk(seed=0, n_envs=1024)
        st = bench.alg_flops(w.name, "step")
        ob = bench.alg_flops(w.name, "observe")
        assert st > 200 and ob >= 11
        assert bench.call_flops(w, 10) == pytest.approx(w.n_quads * (10 * st + ob))
    assert bench.alg_flops("scale_32768x32", "fwdbwd") > bench.alg_flops("scale_32768x32",
                                                                         "rollout")
    assert bench.alg_flops("nonesuch", "step") is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_cpu_baseline_protocol():
    """Median of three runs on every core the process may use and on one
    core, on a bounded sample of the workload; the CPU model is recorded."""
    w = W.custom([8] * 64, seed=0, k=6, name="swarm_4096x8")
    r = bench.cpu_baseline(w, 0.05, n_envs=16, runs=3)
    assert r["kind"] == "oracle" and r["cores"] >= 1
    assert len(r["runs"]) == 3 and r["value"] == pytest.approx(sorted(r["runs"])[1])
    assert r["one_core"]["cores"] == 1 and len(r["one_core"]["runs"]) == 3
    assert r["cpu_model"] and "128 quads" in r["sample"]
