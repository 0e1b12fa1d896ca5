"""Host-side logic of bench.py (CPU only): the algorithmic byte counts, the
gate on stored counter traffic, and the single-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes():
    # pose 12 + occupancy 1 + log-weight 4 + 40 searches x (header 8 + zero point 4)
    # + 21 paired zero points x 4 + 61 table entries x 4
    assert bench.BYTES_PER_PARTICLE == 12 + 1 + 4 + 40 * 12 + 21 * 4 + 61 * 4 == 825
    assert bench.BYTES_PER_CAST == 29
    assert bench.SEARCHES == 40 and bench.RAYS == 61
    # useful bytes per fused ray: header 8 + both bracketing zero points 8 + table entry 4
    # + (pose 12 + occupancy 1 + log-weight 4) / 61
    assert abs(bench.BYTES_PER_RAY_FUSED - 20.2787) < 1e-4


def test_stored_traffic_needs_same_source_particles_and_layout(monkeypatch):
    with open(os.path.join(ROOT, "profiles", "k_batch_traffic.json")) as f:
        stored = json.load(f)
    monkeypatch.setattr(bench, "BUCKETS", stored["layout"]["bucket_log2"])
    monkeypatch.setattr(bench, "ZP16", stored["layout"]["zp16"])
    monkeypatch.setattr(bench, "PRUNE", stored["layout"]["pcddt"])
    if stored["kernel_source_hash"] != bench.kernel_source_hash():
        pytest.skip("kernel source changed since the counters were taken (traffic is then reported as null)")
    assert bench.measured_traffic("k_batch", stored["particles"]) == stored["bytes_per_launch"]
    assert bench.measured_traffic("k_batch", stored["particles"] + 1) is None
    other = 7 if stored["layout"]["bucket_log2"] != 7 else 6
    monkeypatch.setattr(bench, "BUCKETS", other)
    assert bench.measured_traffic("k_batch", stored["particles"]) is None
    monkeypatch.setattr(bench, "BUCKETS", stored["layout"]["bucket_log2"])
    monkeypatch.setattr(bench, "PRUNE", True)
    assert bench.measured_traffic("k_batch", stored["particles"]) is None
    assert bench.measured_traffic("no_such_kernel", stored["particles"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
