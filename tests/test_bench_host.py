"""Host-side logic of bench.py (no GPU): the committed rocprofv3 counter
summaries it reads, the rule that drops them once the kernel source has
changed, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

import bench


@pytest.mark.parametrize("precision", ["f64", "mixed"])
def test_counter_summary_is_consistent(precision):
    """Each kernel's bytes per transported particle are its counted fetch and
    write bytes of one launch over the particles of a step, and the whole
    step's figure is their sum weighted by launches per step (runtime copies
    and init kernels at their fractional rates included); the counters'
    scale factors are positive."""
    with open(bench.TRAFFIC_FILES[precision]) as f:
        t = json.load(f)
    assert len(t["kernel_sha"]) == 16 and int(t["kernel_sha"], 16) >= 0
    assert t["counter_scale"]["FETCH_SIZE"] > 0 and t["counter_scale"]["WRITE_SIZE"] > 0
    n = t["particles_per_step"]
    assert n > 1e6
    total = 0.0
    for name, k in t["kernels"].items():
        per = (k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]) / n
        assert per == pytest.approx(k["bytes_per_particle"], rel=1e-12), name
        total += k["bytes_per_particle"] * k["launches_per_step"]
    assert total == pytest.approx(t["step_bytes_per_particle"], rel=1e-12)
    assert "transport" in t["kernels"] and t["step_bytes_per_particle"] > t["kernels"]["transport"]["bytes_per_particle"]


def test_traffic_is_dropped_when_the_kernels_change(monkeypatch, tmp_path):
    with open(bench.TRAFFIC_FILES["f64"]) as f:
        sha = json.load(f)["kernel_sha"]
    monkeypatch.setattr(bench, "kernel_sha", lambda: sha)
    t = bench.measured_traffic("f64")
    assert t is not None and t["kernel_sha"] == sha
    monkeypatch.setattr(bench, "kernel_sha", lambda: "0" * 16 if sha != "0" * 16 else "1" * 16)
    assert bench.measured_traffic("f64") is None
    monkeypatch.setattr(bench, "TRAFFIC_FILES", {"f64": str(tmp_path / "absent.json")})
    assert bench.measured_traffic("f64") is None


def test_more_than_one_gpu_is_refused():
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU only" in r.stdout + r.stderr
