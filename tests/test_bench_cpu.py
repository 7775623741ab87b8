"""Host logic of bench.py, on the CPU: the one-GPU refusal, the roofline
arithmetic (algorithmic flops over the summed launch time, spec and measured
peaks) and the lookup of recorded counter traffic, which must match the
kernel, the workload and the hash of the current kernel sources."""

import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_arithmetic(monkeypatch):
    monkeypatch.setattr(bench, "recorded_traffic", lambda kernel, workload: None)
    # 4 launches of 25 ms each over 2 steps of 1e12 flops: 2e12 / 0.1 s = 20 TFLOP/s
    prof = {"w_build": (100.0, 4)}
    out = bench.roofline(prof, "w_build", "k", 1e12, 2, 78.6, measured=77.5, workload="w")
    assert out["achieved"] == pytest.approx(20.0)
    assert out["frac"] == pytest.approx(20.0 / 78.6, abs=1e-4)
    assert out["frac_measured"] == pytest.approx(20.0 / 77.5, abs=1e-4)
    assert out["avg_launch_ms"] == pytest.approx(25.0)
    assert out["launches"] == 4 and out["traffic"] is None
    issued = bench.roofline(prof, "w_build", "k", 1e12, 2, 2500.0, issued=3.0)
    assert issued["achieved"] == pytest.approx(60.0)
    assert "3 issued products" in issued["work"]


def test_recorded_traffic_matches_kernel_workload_and_sources(tmp_path, monkeypatch):
    pdir = tmp_path / "profiles"
    pdir.mkdir()
    rec = {"kernel": "k_x", "workload": "w1", "sources_sha256": bench.sources_sha256(),
           "bytes_per_launch": 123, "algorithmic_bytes_per_launch": 100, "launches": 2,
           "profile": "profiles/p.md"}
    stale = dict(rec, workload="w2", sources_sha256="0" * 64)
    (pdir / "p.md").write_text("# p\n\n<!-- traffic: %s -->\n<!-- traffic: %s -->\n"
                               % (json.dumps(rec), json.dumps(stale)))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "sources_sha256", lambda: rec["sources_sha256"])
    assert bench.recorded_traffic("k_x", "w1") == rec
    assert bench.recorded_traffic("k_x", "w2") is None       # taken with other sources
    assert bench.recorded_traffic("k_y", "w1") is None
    monkeypatch.setattr(bench, "recorded_traffic", lambda kernel, workload: rec)
    out = bench.roofline({"c": (10.0, 2)}, "c", "k_x", 1e9, 1, 78.6, workload="w1")
    assert out["traffic"] == 123 and out["algorithmic_bytes"] == 100


def test_sources_hash_covers_every_kernel_source():
    csrc = os.path.join(ROOT, "paper_2412_18553_amd", "csrc")
    names = sorted(os.listdir(csrc))
    assert any(n.endswith(".hip") for n in names) and any(n.endswith(".hpp") for n in names)
    h = bench.sources_sha256()
    assert len(h) == 64 and h == bench.sources_sha256()


@pytest.mark.parametrize("mode,prec", [("fp64", "split_bf16"), ("split", "fp64"),
                                       ("projector", "split_bf16"), ("df", "fp64")])
def test_fixed_precision_modes_refuse_another(mode, prec):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mode", mode,
                        "--precision", prec], capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert f"--mode {mode} runs in" in r.stderr
    assert r.stdout == ""
