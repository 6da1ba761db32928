"""Summaries of rocprofv3 runs of bench.py (the figures under profiles/).

    python profile_report.py trace <run dir> <groups> [--skip S]
    python profile_report.py hbm   <run dir> <groups> [--skip S] [--write-traffic WORKLOAD]
    python profile_report.py mfma  <run dir> <groups> [--skip S]

<run dir> is the -d folder of one rocprofv3 run (--kernel-trace for trace,
--pmc for hbm and mfma).  The window is <groups> slice groups, each ending at
a k_accumulate: the last <groups> of the run, or, with --skip S, the ones
after the first S (0 groups = every dispatch).

trace: kernel time per kernel and per roofline class in the window.

hbm: bytes per launch from the TCC_EA0 request counters and their request
sizes, read = (RDREQ - RDREQ_32B) x 128 + RDREQ_32B x 32 and written =
WRREQ_64B x 64 + (WRREQ - WRREQ_64B) x 32 (on a plain 1 GiB device copy these
give 1 GiB read and 1 GiB written per launch).  With --write-traffic, also
writes profiles/traffic_<class>.json, the per-launch HBM bytes of each kernel
class that bench.py reports as roofline.traffic for that workload key and the
current library sources.

mfma: matrix-core busy fraction and MFMA flops per kernel from
SQ_VALU_MFMA_BUSY_CYCLES, SQ_INSTS_VALU_MFMA_MOPS_* and GRBM_GUI_ACTIVE.
"""
import argparse
import collections
import csv
import glob
import json
import os
import re

ROOT = os.path.dirname(os.path.abspath(__file__))
XCC, SIMD, CLK = 8, 1024, 2.4e9  # XCDs, SIMDs, clock of an MI355X
FP32_PEAK, HALF_PEAK = 157.3e12, 2516.6e12

# kernel classes of the roofline: members (whose bytes count) and the launches
# that count as one op (the long contraction's partial-sum pass belongs to its op)
CLASSES = {
    "stream": (lambda n: n.startswith("k_stream"),
               lambda n: n.startswith("k_stream") and not n.startswith("k_stream_lk_sum")),
    "gemm": (lambda n: n.startswith("k_cgemm") or n.startswith("k_gemm_ksum"), lambda n: n.startswith("k_cgemm")),
    "permute": (lambda n: n.startswith("k_permute"), lambda n: n.startswith("k_permute")),
}


def short(name):
    name = re.sub(r"\(.*", "", name)
    return name.replace("void rqc::", "").replace("rqc::", "").strip()


def trace(d):
    f = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    rs = list(csv.DictReader(open(f)))
    rs.sort(key=lambda r: int(r["Start_Timestamp"]))
    return [{"name": short(r["Kernel_Name"]), "start": int(r["Start_Timestamp"]), "end": int(r["End_Timestamp"])}
            for r in rs]


def dispatches(d):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    disp = collections.OrderedDict()
    for r in csv.DictReader(open(f)):
        e = disp.setdefault(int(r["Dispatch_Id"]), {"name": short(r["Kernel_Name"])})
        e[r["Counter_Name"]] = e.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    return [disp[k] for k in sorted(disp)]


def window(rs, groups, skip=None):
    if groups <= 0:
        return rs
    acc = [i for i, r in enumerate(rs) if r["name"] == "k_accumulate"]
    if skip is None:
        start = acc[-groups - 1] + 1 if len(acc) > groups else 0
        return rs[start:acc[-1] + 1]
    start = acc[skip - 1] + 1 if skip > 0 else 0
    return rs[start:acc[skip + groups - 1] + 1]


def class_of(name):
    for cls, (member, _) in CLASSES.items():
        if member(name):
            return cls
    return "other"


def kernel_times(rs, groups):
    stat = collections.defaultdict(lambda: [0, 0.0])
    for r in rs:
        stat[r["name"]][0] += 1
        stat[r["name"]][1] += (r["end"] - r["start"]) / 1e3
    tot = sum(t for _, t in stat.values())
    wall = (rs[-1]["end"] - rs[0]["start"]) / 1e6
    print(f"timed window: {groups} slice groups, kernel time {tot / 1e3:.1f} ms, first start to last end "
          f"{wall:.1f} ms")
    print(f"  {'kernel':44s} {'calls':>6s} {'total ms':>10s} {'avg us':>10s} {'share':>6s}")
    for k, (n, t) in sorted(stat.items(), key=lambda x: -x[1][1])[:24]:
        print(f"  {k:44s} {n:6d} {t / 1e3:10.2f} {t / n:10.1f} {100 * t / tot:5.1f}%")
    cls = collections.defaultdict(lambda: [0, 0.0])
    for k, (n, t) in stat.items():
        c = class_of(k)
        cls[c][1] += t
        if c != "other" and CLASSES[c][1](k):
            cls[c][0] += n
    for c, (n, t) in sorted(cls.items(), key=lambda x: -x[1][1]):
        print(f"class {c}: " + (f"{n} ops, " if n else "") + f"{t / 1e3:.2f} ms" +
              (f", {t / n:.1f} us per op" if n else ""))


def read_bytes(r):
    return (r["TCC_EA0_RDREQ_sum"] - r["TCC_EA0_RDREQ_32B_sum"]) * 128 + r["TCC_EA0_RDREQ_32B_sum"] * 32


def write_bytes(r):
    return r["TCC_EA0_WRREQ_64B_sum"] * 64 + (r["TCC_EA0_WRREQ_sum"] - r["TCC_EA0_WRREQ_64B_sum"]) * 32


def per_kernel(rs):
    agg = collections.OrderedDict()
    for r in rs:
        a = agg.setdefault(r["name"], collections.defaultdict(float))
        a["n"] += 1
        for k, v in r.items():
            if k != "name":
                a[k] += v
    return agg


def hbm(rs, workload):
    agg = per_kernel(rs)
    print(f"  {'kernel':34s} launches  read GiB/launch  written GiB/launch")
    for k, a in sorted(agg.items(), key=lambda x: -(read_bytes(x[1]) + write_bytes(x[1]))):
        n = a["n"]
        print(f"  {k:34s} {int(n):6d}  {read_bytes(a) / n / 2**30:15.4f}  {write_bytes(a) / n / 2**30:18.4f}")
    if workload is None:
        return
    import bench
    for cls, (member, counted) in CLASSES.items():
        b = sum(read_bytes(r) + write_bytes(r) for r in rs if member(r["name"]))
        n = sum(1 for r in rs if counted(r["name"]))
        if n == 0:
            continue
        rec = {"kernel_class": cls, "bytes_per_launch": b / n, "launches_counted": n,
               "read_bytes_per_request": 128, "read_bytes_per_32b_request": 32,
               "write_bytes_per_64b_request": 64, "write_bytes_per_other_request": 32,
               "counters": ["TCC_EA0_RDREQ_sum", "TCC_EA0_RDREQ_32B_sum", "TCC_EA0_WRREQ_sum",
                            "TCC_EA0_WRREQ_64B_sum"],
               "copy_check": "a 1 GiB device copy reads 1.0000 GiB and writes 1.0000 GiB by these request sizes",
               "source_sha256": bench.source_sha256(), "workload": workload,
               "sources": list(bench.TRAFFIC_SOURCES)}
        with open(os.path.join(ROOT, "profiles", f"traffic_{cls}.json"), "w") as f:
            json.dump(rec, f, indent=1)
        print(f"{cls}: {n} ops, {b / n / 1e6:.1f} MB per op")


def mfma(rs):
    for k, a in sorted(per_kernel(rs).items(), key=lambda x: -x[1]["SQ_VALU_MFMA_BUSY_CYCLES"]):
        if a["SQ_VALU_MFMA_BUSY_CYCLES"] <= 0:
            continue
        cyc = a["GRBM_GUI_ACTIVE"] / XCC
        util = a["SQ_VALU_MFMA_BUSY_CYCLES"] / (cyc * SIMD)
        f32 = a["SQ_INSTS_VALU_MFMA_MOPS_F32"] * 512
        half = (a["SQ_INSTS_VALU_MFMA_MOPS_BF16"] + a["SQ_INSTS_VALU_MFMA_MOPS_F16"]) * 512
        t = cyc / CLK
        print(f"  {k:34s} launches {int(a['n']):4d}  MFMA busy {100 * util:5.1f}%  "
              f"FP32 {f32 / a['n'] / 1e9:9.2f} GFLOP/launch ({f32 / t / 1e12:6.1f} TFLOP/s = "
              f"{100 * f32 / t / FP32_PEAK:5.1f}% of 157.3)  bf16/fp16 {half / a['n'] / 1e9:9.2f} GFLOP/launch "
              f"({half / t / 1e12:7.1f} TFLOP/s = {100 * half / t / HALF_PEAK:5.1f}% of 2516.6)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=("trace", "hbm", "mfma"))
    ap.add_argument("run_dir")
    ap.add_argument("groups", type=int)
    ap.add_argument("--skip", type=int, default=None, help="slice groups before the window, from the start")
    ap.add_argument("--write-traffic", default=None, metavar="WORKLOAD")
    a = ap.parse_args()
    if a.kind == "trace":
        kernel_times(window(trace(a.run_dir), a.groups, a.skip), a.groups)
        return
    rs = window(dispatches(a.run_dir), a.groups, a.skip)
    if a.kind == "hbm":
        hbm(rs, a.write_traffic)
    else:
        mfma(rs)


if __name__ == "__main__":
    main()
