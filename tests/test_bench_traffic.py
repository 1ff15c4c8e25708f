"""The benchmark's host logic (CPU): the counted-traffic lookup (the committed rocprofv3 HBM summary
is reported only for the kernel, precision and delay depth it was taken at, and only while the
downdate's source is the one profiled), the roofline arithmetic, and the one-GPU refusal."""
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


def test_roofline_fields_from_a_profile():
    """The roofline object's arithmetic on a made-up profile: 1e13 algorithmic flops and 4e11 bytes
    over 4 launches in 100 ms."""
    prof = {"ms": {"syrk": 100.0}, "launches": {"syrk": 4}, "syrk_flops": 1.0e13, "syrk_bytes": 4.0e11}
    r = bench.roofline_syrk(prof, "mixed_f32")
    assert r["bound"] == "mfma" and r["unit"] == "TFLOP/s" and r["peak"] == 157.3
    assert abs(r["achieved"] - 100.0) < 1e-9 and abs(r["frac"] - round(100.0 / 157.3, 4)) < 1e-12
    assert r["avg_launch_ms"] == 25.0 and r["algorithmic_bytes_per_launch"] == 1.0e11
    assert abs(r["algorithmic_gbs"] - 4000.0) < 1e-6 and r["traffic"] is None
    b = bench.roofline_syrk(prof, "mixed_bf16x3")
    # three BF16 products per algorithmic one: reported against the HBM peak, the executed BF16
    # rate beside it
    assert b["bound"] == "hbm" and b["unit"] == "GB/s" and abs(b["achieved"] - 4000.0) < 1e-6
    assert abs(b["executed_bf16_tflops"] - 300.0) < 1e-9 and abs(b["bf16_mfma_frac"] - 0.12) < 1e-12


def test_more_than_one_gpu_is_refused():
    import subprocess
    import sys
    p = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr
