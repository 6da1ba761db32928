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


def _rec(cls, seconds, flops, bytes_, exec_flops, kind=0, launches=1, op=0):
    return {"cls": cls, "op": op, "launches": launches, "seconds": seconds, "flops": flops, "bytes": bytes_,
            "exec_flops": exec_flops, "exec_kind": kind}


def _ops(gemm_s, stream_s, kind=0):
    g_exec = 8e12 * (6.0 / 8.0 if kind == 0 else 3.0)
    return [
        _rec("gemm", gemm_s, 8e12, 4e9, g_exec, kind, launches=4, op=1),
        # two streaming ops: one HBM-bound, one bound by its matrix-core stages
        _rec("stream", 0.5 * stream_s, 0.1e12, 3.9e12, 0.1e12, launches=4, op=2),
        _rec("stream", 0.5 * stream_s, 0.9e12, 0.1e12, 0.9e12, launches=4, op=3),
        _rec("sample", 10.0, 0.0, 0.0, 0.0, op=-1),  # never the dominant class
    ]


def test_gemm_roofline_counts_executed_matrix_core_flops():
    r = bench.kernel_roofline(_ops(1.0, 0.5))
    # 8e12 flops counted at 8 per complex multiply-add = 1e12 multiply-adds,
    # 6 executed flops each on the FP32 matrix cores (three real products)
    assert r["kernel"] == "gemm" and r["bound"] == "mfma" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(6.0)
    assert r["peak"] == 157.3 and r["frac"] == pytest.approx(6.0 / 157.3)
    assert r["binding_frac"] == pytest.approx(6.0 / 157.3)
    assert r["avg_launch_us"] == pytest.approx(0.25e6)
    assert r["bytes_per_launch"] == pytest.approx(1e9)
    r = bench.kernel_roofline(_ops(1.0, 0.5, kind=1))
    # split precision: three half-precision products per real product
    assert r["achieved"] == pytest.approx(24.0) and r["peak"] == 2516.6


def test_stream_roofline_binds_per_op():
    r = bench.kernel_roofline(_ops(0.5, 1.0))
    assert r["kernel"] == "stream"
    # per op: 3.9e12 B / 8 TB/s = 0.4875 s; the second op: max(0.9e12 flop /
    # 157.3 TFLOP/s, 0.1e12 B / 8 TB/s) = 12.5 ms
    tmin = 3.9e12 / 8e12 + max(0.9e12 / 157.3e12, 0.1e12 / 8e12)
    assert r["binding_frac"] == pytest.approx(tmin / 1.0)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved"] == pytest.approx(4000.0) and r["frac"] == pytest.approx(0.5)
    assert r["mfma_side"]["achieved"] == pytest.approx(1.0)
    assert r["launches"] == 8 and r["bytes_per_launch"] == pytest.approx(5e11)
    assert r["traffic"] is None  # no plan named
    # the class whose minimum time is mostly matrix-core time reports that roof
    ops = [_rec("stream", 1.0, 1e14, 1e11, 1e14), _rec("gemm", 0.1, 1e9, 1e6, 1e9)]
    r = bench.kernel_roofline(ops)
    assert r["bound"] == "mfma" and r["frac"] == pytest.approx(100.0 / 157.3)


def test_path_roofline_sums_per_op_minimum_times():
    ops = _ops(1.0, 0.5)
    r = bench.path_roofline(ops, 2.0)
    t = max(8e12 / 157.3e12, 4e9 / 8e12) + max(0.1e12 / 157.3e12, 3.9e12 / 8e12) + \
        max(0.9e12 / 157.3e12, 0.1e12 / 8e12)
    assert r["tmin_seconds"] == pytest.approx(t) and r["frac"] == pytest.approx(t / 2.0)


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


def test_gate_count_of_the_53_qubit_circuit():
    """The CPU baseline scales its per-gate time by the 53-qubit circuit's gate
    count, taken from the oracle's parser (its state vector code refuses
    circuits that wide)."""
    import synthetic
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    lines = [ln.split() for ln in text.splitlines()]
    want = sum(1 for w in lines if w and w[0] in ("sx", "sy", "sw", "fsim"))
    assert bench.gate_count(text) == want > 1000


def test_serving_workload_text_follows_the_parameters():
    """The serving line's workload string is built from the parameters the run
    uses (shapes, cycles, amplitudes, samples, precision mix, cost cap)."""
    kw = dict(bench.SERVE_KW)
    text = bench.serve_workload_text(1000, kw, bench.SERVE_CAP)
    qubits = sorted(r * c for r, c in kw["shapes"])
    assert f"{qubits[0]}..{qubits[-1]} qubits" in text and "20..40 qubits" in text
    assert f"{kw['cycles'][0]}..{kw['cycles'][1]} cycles" in text and "8..20 cycles" in text
    assert f"2^{kw['log2_amps'][0]}..2^{kw['log2_amps'][1]} amplitudes" in text
    assert f"{kw['samples'][0]}..{kw['samples'][1]} samples" in text
    assert text.startswith("serving: 1000 seeded requests per load")
    kw["cycles"] = (3, 5)
    assert "3..5 cycles" in bench.serve_workload_text(10, kw, 1e9)
