"""Host-side logic of the benchmark script (no GPU): the one-GPU guard, and the scaling
of the committed counter summary's HBM traffic to a run's own launch size."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus"] == 2


def _summary(tmp_path, **rec):
    os.makedirs(tmp_path / "profiles", exist_ok=True)
    with open(tmp_path / "profiles" / "pmc_fused_pass_t.json", "w") as fh:
        json.dump(rec, fh)


def test_traffic_scales_with_the_launch_and_needs_the_same_sources(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    # the same launch size gives the measured bytes back; twice the algorithmic bytes, twice
    _summary(tmp_path, kernel_source_hash=h, bytes_per_launch=950, bytes_alg_per_launch=1000.0)
    assert bench.traffic_from_profiles("t", 1000.0) == 950
    assert bench.traffic_from_profiles("t", 2000.0) == 1900
    # counters taken on other sources, or without the counted run's size, are not used
    _summary(tmp_path, kernel_source_hash="other", bytes_per_launch=950, bytes_alg_per_launch=1000.0)
    assert bench.traffic_from_profiles("t", 1000.0) is None
    _summary(tmp_path, kernel_source_hash=h, bytes_per_launch=950)
    assert bench.traffic_from_profiles("t", 1000.0) is None
    assert bench.traffic_from_profiles("missing", 1000.0) is None
