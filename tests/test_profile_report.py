"""CPU tests of profile_report.py, the script that turns rocprofv3 CSVs into
the tables under profiles/ and the per-class traffic records bench.py reads:
the timed window (last groups, or groups after a skip), bytes from request
counts and sizes, per-class op counts (the long contraction's partial-sum
pass is not an op of its own), and the traffic record's fields."""
import csv
import importlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
pr = importlib.import_module("profile_report")


def _trace(tmp_path, names):
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "x_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        t = 1000
        for n, dur in names:
            w.writerow({"Kernel_Name": n, "Start_Timestamp": t, "End_Timestamp": t + dur})
            t += dur + 500
    return str(d)


def _counters(tmp_path, rows):
    d = tmp_path / "pmc"
    d.mkdir()
    with open(d / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (n, ctr) in enumerate(rows):
            for k, v in ctr.items():
                # two XCD rows per counter: the script adds them
                w.writerow({"Dispatch_Id": i, "Kernel_Name": n, "Counter_Name": k, "Counter_Value": v / 2})
                w.writerow({"Dispatch_Id": i, "Kernel_Name": n, "Counter_Name": k, "Counter_Value": v / 2})
    return str(d)


GROUP = [("void rqc::k_cgemm_f32<128, 128, 0, 1>(rqc::GemmArgs)", 3000),
         ("void rqc::k_stream_lk<4>(float2 const*)", 2000),
         ("rqc::k_stream_lk_sum(float2 const*)", 100),
         ("rqc::k_permute(rqc::PermDesc const*)", 400),
         ("rqc::k_accumulate(float2 const*)", 50)]


def test_window_and_kernel_times(tmp_path, capsys):
    names = [("rqc::k_norm(float2 const*)", 10)] + GROUP * 4
    rs = pr.trace(_trace(tmp_path, names))
    assert [r["name"] for r in rs[:2]] == ["k_norm", "k_cgemm_f32<128, 128, 0, 1>"]
    last2 = pr.window(rs, 2)
    assert len(last2) == 2 * len(GROUP) and last2[-1]["name"] == "k_accumulate"
    mid = pr.window(rs, 2, skip=1)
    assert len(mid) == 2 * len(GROUP) and mid[0] is rs[1 + len(GROUP)]
    assert pr.window(rs, 0) is rs
    pr.kernel_times(last2, 2)
    out = capsys.readouterr().out
    # gemm: 2 ops of 3 us; stream: 2 ops, each with its partial-sum pass time
    assert "class gemm: 2 ops, 0.01 ms, 3.0 us per op" in out
    assert "class stream: 2 ops, 0.00 ms, 2.1 us per op" in out
    assert "class permute: 2 ops" in out and "class other: 0.00 ms" in out


def test_request_bytes():
    r = {"TCC_EA0_RDREQ_sum": 10.0, "TCC_EA0_RDREQ_32B_sum": 4.0, "TCC_EA0_WRREQ_sum": 7.0,
         "TCC_EA0_WRREQ_64B_sum": 5.0}
    assert pr.read_bytes(r) == 6 * 128 + 4 * 32
    assert pr.write_bytes(r) == 5 * 64 + 2 * 32


def test_traffic_record(tmp_path, monkeypatch, capsys):
    ctr = {"TCC_EA0_RDREQ_sum": 8.0, "TCC_EA0_RDREQ_32B_sum": 0.0, "TCC_EA0_WRREQ_sum": 4.0,
           "TCC_EA0_WRREQ_64B_sum": 4.0}
    rows = [(n, ctr) for n, _ in GROUP] * 3
    rs = pr.window(pr.dispatches(_counters(tmp_path, rows)), 2)
    assert len(rs) == 2 * len(GROUP)
    out_dir = tmp_path / "root"
    (out_dir / "profiles").mkdir(parents=True)
    monkeypatch.setattr(pr, "ROOT", str(out_dir))
    pr.hbm(rs, "mid:c64:full:tree=0")
    per_dispatch = 8 * 128 + 4 * 64
    rec = json.load(open(out_dir / "profiles" / "traffic_stream.json"))
    # two lk launches and two partial-sum passes over two lk ops
    assert rec["launches_counted"] == 2 and rec["bytes_per_launch"] == 2 * per_dispatch
    assert rec["workload"] == "mid:c64:full:tree=0" and len(rec["source_sha256"]) == 64
    g = json.load(open(out_dir / "profiles" / "traffic_gemm.json"))
    assert g["launches_counted"] == 2 and g["bytes_per_launch"] == per_dispatch
    assert "k_permute" in capsys.readouterr().out
