"""The bench attaches measured HBM traffic only to the kernel, mode and
workload the committed counter record was taken on (no GPU)."""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import bench  # noqa: E402


def test_record_is_not_applied_to_other_kernels_modes_or_sizes():
    assert bench.traffic_record("gradient", 1024, 256, deterministic=True) is None
    assert bench.traffic_record("hvp", 1024, 256) is None
    assert bench.traffic_record("gradient", 512, 256) is None
    assert bench.traffic_record("gradient", 1024, 128) is None


def test_record_follows_the_kernel_sources(monkeypatch):
    rec = bench.traffic_record("gradient", 1024, 256)
    if rec is not None:
        assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes"] + rec["write_bytes"] > 0
    monkeypatch.setattr(bench, "kernel_sources_sha256", lambda: "0" * 64)
    assert bench.traffic_record("gradient", 1024, 256) is None
