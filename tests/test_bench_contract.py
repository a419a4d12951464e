"""Host-side pieces of the benchmark contract (CPU): the single-GPU refusal,
the HBM traffic figure taken from the committed rocprofv3 counter summary
only while it matches the current kernel source, and the kernel names the
roofline entry reports."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

TRAFFIC = os.path.join(ROOT, "profiles", "stream_collide_c2_dense_traffic.json")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_only_for_the_current_kernel_source(monkeypatch):
    with open(TRAFFIC) as fh:
        d = json.load(fh)
    if d["kernel_hash"] != bench.kernel_hash():
        pytest.skip("the counter summary predates the current stream-collide source")
    assert bench.traffic_from_profiles(0) == d["bytes_per_launch"]["0"]
    assert bench.traffic_from_profiles(1) == d["bytes_per_launch"]["1"]
    assert bench.traffic_from_profiles(2) == d["bytes_per_launch"]["2"]
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0" * 16)
    assert bench.traffic_from_profiles(0) is None


def test_traffic_summary_is_consistent():
    with open(TRAFFIC) as fh:
        d = json.load(fh)
    ncell = 256 ** 3
    for key, bpc in (("0", 152), ("1", 76), ("2", 76)):
        e = d["by_storage"][key]
        assert e["algorithmic_bytes_per_launch"] == bpc * ncell
        total = e["read_bytes_per_launch"] + e["write_bytes_per_launch"]
        assert total == d["bytes_per_launch"][key]
        # HBM bytes cannot fall short of what the kernel must move
        assert 1.0 <= total / e["algorithmic_bytes_per_launch"] < 1.5
        cal = e["calibration"]
        assert cal["known_KiB_each_direction"] == bpc * ncell / 2 / 1024


def test_roofline_kernel_names():
    assert bench.stream_collide_kernel(0, 256) == "k_stream_collide"
    assert bench.stream_collide_kernel(1, 256) == "k_stream_collide_pairs"
    assert bench.stream_collide_kernel(2, 128) == "k_stream_collide_pairs"
    assert bench.stream_collide_kernel(1, 13) == "k_stream_collide"
    assert bench.BYTES_PER_CELL == {0: 152, 1: 76, 2: 76}
