"""The benchmark's counted-traffic lookup (CPU): the committed rocprofv3 HBM summary is reported
only for the kernel, precision and delay depth it was taken at, and only while the downdate's
source is the one profiled."""
import json
import os

import pytest

import bench

WL = "mixed_600x128"


def test_committed_summary_is_consistent_and_found():
    path = os.path.join(bench.ROOT, "profiles", f"syrk_hbm_traffic_{WL}.json")
    with open(path) as fh:
        rec = json.load(fh)
    for prec, kernel in bench.SYRK_KERNEL.items():
        ent = rec["kernels"][prec]
        assert ent["kernel"] == kernel
        for row in ent["by_delay"].values():
            assert abs(row["hbm_bytes_per_launch"] - row["fetch_bytes_per_launch"] - row["write_bytes_per_launch"]) <= 1
            assert row["hbm_bytes_per_launch"] >= 0.99 * row["algorithmic_bytes_per_launch"]
    if any(rec["kernels"][p]["source_sha256"] != bench.source_digest() for p in bench.SYRK_KERNEL):
        pytest.skip("the downdate's source changed since the counters were taken: the benchmark reports no traffic")
    for prec, kernel in bench.SYRK_KERNEL.items():
        for d, row in rec["kernels"][prec]["by_delay"].items():
            assert bench.counted_traffic(WL, prec, kernel, int(d)) == row["hbm_bytes_per_launch"]


def test_lookup_refuses_other_delay_kernel_workload_or_source(monkeypatch):
    kernel = bench.SYRK_KERNEL["mixed_f32"]
    assert bench.counted_traffic(WL, "mixed_f32", kernel, 1) is None          # depth not profiled
    assert bench.counted_traffic(WL, "mixed_f32", "other_kernel", 4) is None  # other kernel
    assert bench.counted_traffic("no_such_workload", "mixed_f32", kernel, 4) is None
    monkeypatch.setattr(bench, "source_digest", lambda: "0" * 64)            # source changed
    assert bench.counted_traffic(WL, "mixed_f32", kernel, 4) is None
