"""Host logic of bench.py (no GPU): the roofline arithmetic on a made-up
profile, the refusal of more than one GPU, and that a committed HBM-traffic
record is reported only for the plan and library sources it was taken on."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _prof(gemm_s, stream_s):
    return {
        "gemm": {"seconds": gemm_s, "flops": 8e12, "bytes": 4e9, "launches": 4},
        "stream": {"seconds": stream_s, "flops": 1e12, "bytes": 4e12, "launches": 8},
        "sample": {"seconds": 10.0, "flops": 0.0, "bytes": 0.0, "launches": 1},  # never the dominant class
    }


def test_gemm_roofline_counts_executed_matrix_core_flops():
    r = bench.kernel_roofline(_prof(1.0, 0.5), True)
    # 8e12 flops counted at 8 per complex multiply-add = 1e12 multiply-adds,
    # 6 executed flops each on the FP32 matrix cores (three real products)
    assert r["kernel"] == "gemm" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(6.0)
    assert r["peak"] == 157.3 and r["frac"] == pytest.approx(6.0 / 157.3)
    assert r["avg_launch_us"] == pytest.approx(0.25e6)
    assert r["bytes_per_launch"] == pytest.approx(1e9)
    r = bench.kernel_roofline(_prof(1.0, 0.5), False)
    # split precision: three half-precision products per real product
    assert r["achieved"] == pytest.approx(24.0) and r["peak"] == 2516.6


def test_stream_roofline_is_hbm_bound_with_matrix_core_side():
    r = bench.kernel_roofline(_prof(0.5, 1.0), True)
    assert r["kernel"] == "stream" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    assert r["mfma_side"]["achieved"] == pytest.approx(1.0)
    assert r["launches"] == 8 and r["bytes_per_launch"] == pytest.approx(5e11)
    assert r["traffic"] is None  # no plan named


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr and p.stdout == ""


@pytest.mark.parametrize("cls", ["gemm", "stream"])
def test_traffic_record_only_for_its_plan(cls):
    rec = json.load(open(os.path.join(ROOT, "profiles", f"traffic_{cls}.json")))
    key = rec["workload"]
    assert key.startswith("mid:c64:full:tree=")
    got = bench.measured_traffic(cls, key)
    if rec["source_sha256"] == bench.source_sha256():
        assert got == rec["bytes_per_launch"]
    else:
        assert got is None  # sources changed since the counters were taken
    assert bench.measured_traffic(cls, key.replace("tree=", "tree=x")) is None
    assert bench.measured_traffic(cls, key.replace("mid:", "tiny:")) is None
    assert bench.measured_traffic(cls, None) is None
