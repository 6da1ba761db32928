"""Throughput of the sliced-contraction sampler on one MI355X.

One step = one open batch of amplitudes through the whole hot path: leaf
selection per slice group, the contraction program (fused small subtrees,
streaming contractions, permutes, MFMA complex GEMMs), the FP64 cross-slice
sum, normalisation, and rejection sampling over the batch's sub-batches of 64.
Fixed output bits are fresh per step (seeded).  Prints one JSON line; its
"global_cache" object times the same steps again on a plan that keeps the
fixed-bit-independent parts of the contraction per slice group (the headline
value recomputes everything every step).

Workloads:
  mid (default)  5x6 grid, 14 cycles, 6 sliced legs (64 slices), 2^12 batch
  precision      5x6 grid, 16 cycles, 10 sliced legs (1024 slices), 2^14 batch,
                 in complex64 / bf16x3 / fp16x3 (--precision)
  large          53 qubits (6x9 minus (0,4)), 20 cycles: one GPU's share (2^10
                 slices) of a contraction sliced to 2^30-element intermediates,
                 timed on a prefix of the slice list and extrapolated (labelled)
  --serve        the serving loop on a Poisson stream of synthetic requests
  --copy-calibration  a plain 1 GiB device copy, for scaling HBM counters

Plans come from a 65536-trial tree search whose 4 best estimated trees are
timed on the GPU (--path-trials, --autotune); planning is reported separately
(plan_seconds) and is not part of a step.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402

PEAK = {"fp32_mfma_tflops": 157.3, "bf16_mfma_tflops": 2516.6, "hbm_gbs": 8000.0}
METRIC = "contraction TFLOP/s + amplitudes/s at stated error vs FP64; p50/p99 latency"
N_SLICED = {"tiny": 0, "mid": 6, "precision": 10}
DTYPE = {"c64": "complex64 (fp32 MFMA), fp64 slice sum",
         "bf16x3": "bf16x3 split (bf16 MFMA, fp32 acc), fp64 slice sum",
         "fp16x3": "fp16x3 split with 2^e scaling (fp16 MFMA, fp32 acc), fp64 slice sum"}


def cpu_baseline(cfg, text, budget_s=20.0):
    """The oracle's FP64 state vector timed on a bounded prefix of the gate list,
    extrapolated to the whole circuit; returns requested-amplitudes/s."""
    from oracle import sv as osv
    n = osv.num_qubits(text)
    n_gates = osv.num_gates(text)
    threads = osv.max_threads()
    buf = np.empty(1 << n, dtype=np.complex128)
    t0 = time.perf_counter()
    osv.simulate(text, max_gates=0, out=buf)
    t_init = time.perf_counter() - t0
    g = 4
    while True:
        t0 = time.perf_counter()
        osv.simulate(text, max_gates=g, out=buf)
        dt = time.perf_counter() - t0 - t_init
        if dt * 2 > budget_s or g >= n_gates:
            break
        g = min(n_gates, g * 2)
    per_gate = max(dt, 1e-9) / g
    t_full = t_init + per_gate * n_gates
    amps = 1 << len(cfg["open_qubits"])
    return {"value": amps / t_full, "unit": "amplitudes/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 state vector of {n} qubits over the first {g} of {n_gates} gates "
                      f"({dt:.1f} s), extrapolated linearly to the full circuit ({t_full:.0f} s per "
                      f"{amps}-amplitude batch; it also yields the other 2^{n - len(cfg['open_qubits'])}"
                      f" batches)"}


# real matrix-core flops per complex multiply-add: the FP32 GEMM takes three
# real products (Gauss), the split GEMMs three bf16/fp16 products of the 2K-long
# interleaved real view for each of the real and imaginary outputs
MFMA_FLOPS_PER_CMAC = {True: 6.0, False: 24.0}


def kernel_roofline(prof, precision_is_c64, workload=None):
    """Dominant kernel class by measured time and its achieved fraction."""
    cls = max((k for k in prof if k != "sample"), key=lambda k: prof[k]["seconds"])
    pc = prof[cls]
    if cls == "gemm":
        peak = PEAK["fp32_mfma_tflops"] if precision_is_c64 else PEAK["bf16_mfma_tflops"]
        # pc["flops"] counts 8 per complex multiply-add; the matrix cores execute
        # MFMA_FLOPS_PER_CMAC of them
        achieved = pc["flops"] * MFMA_FLOPS_PER_CMAC[precision_is_c64] / 8.0 / pc["seconds"] / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                "flops_per_complex_mac": MFMA_FLOPS_PER_CMAC[precision_is_c64],
                "complex_tflops_8_per_mac": pc["flops"] / pc["seconds"] / 1e12}
    else:
        achieved = pc["bytes"] / pc["seconds"] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm_gbs"]}
        if cls == "stream" and pc["flops"] > 0:
            # the streaming contractions run their multiply on the FP32 matrix
            # cores as real block products (8 real flops per complex
            # multiply-add, as counted); fused pairs and long contractions make
            # that side a bound too
            mf = pc["flops"] / pc["seconds"] / 1e12
            roof["mfma_side"] = {"achieved": mf, "peak": PEAK["fp32_mfma_tflops"], "unit": "TFLOP/s",
                                 "frac": mf / PEAK["fp32_mfma_tflops"]}
    roof.update({"kernel": cls, "launches": pc["launches"],
                 "avg_launch_us": 1e6 * pc["seconds"] / max(1, pc["launches"]),
                 "bytes_per_launch": pc["bytes"] / max(1, pc["launches"]),
                 "traffic": measured_traffic(cls, workload)})
    return roof


def source_sha256():
    """One digest over the library sources (kernels and the lowering that
    decides their tiles and layouts both change the traffic)."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_15083_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".cpp", ".hpp")):
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()


def tree_digest(rqc, plan):
    """Short digest of a plan's contraction tree and sliced legs: the autotune
    may keep a different tree on another run."""
    tree = json.dumps([rqc.plan_path(plan), rqc.plan_sliced_legs(plan)])
    return hashlib.sha256(tree.encode()).hexdigest()[:16]


def traffic_key(args, tree):
    """The plan a counter record belongs to: workload, precision, slicing and
    the contraction tree."""
    return f"{args.config}:{args.precision}:{'partial' if args.target_fidelity else 'full'}:tree={tree}"


def measured_traffic(cls, workload):
    """HBM traffic per launch from the committed counter summary, if it was taken
    on this workload and the current library source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{cls}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_sha256") != source_sha256() or rec.get("workload") != workload:
        return None
    return rec.get("bytes_per_launch")


def run_mid_like(args, rqc, torch):
    torch.cuda.set_device(0)
    cfg = synthetic.CONFIGS[args.config]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    o = len(open_q)
    prec = {"c64": rqc.C64, "bf16x3": rqc.BF16X3, "fp16x3": rqc.FP16X3}[args.precision]
    circ = rqc.load_circuit(text)
    t0 = time.perf_counter()
    partial = {}
    if args.target_fidelity:
        partial = dict(target_fidelity=args.target_fidelity)
    n_sliced = args.partial_sliced if args.target_fidelity else N_SLICED[args.config]
    plan = rqc.plan_create(circ, open_q, n_sliced_target=n_sliced, path_trials=args.path_trials,
                           path_seed=args.path_seed, precision=prec, profile=1, autotune=args.autotune, **partial)
    plan_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    stream = torch.cuda.current_stream()
    out = torch.empty((1, 1 << o, 2), dtype=torch.float32, device="cuda")
    out64 = torch.empty((1, 1 << o, 2), dtype=torch.float64, device="cuda")
    samples = torch.zeros(1 << (o - 6), dtype=torch.int64, device="cuda")
    alpha = cfg["alpha"]

    def step(i, record=None, pl=None):
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + i)]
        rqc.contract_amplitudes(pl or plan, fb, out, out64, stream=stream)
        n_out, st, _ = rqc.rejection_sample(out, fb, open_q, n, samples.numel(), samples, alpha=alpha,
                                            F_norm=1.0, seed=synthetic.SAMPLER_SEED,
                                            batch_index_base=i << (o - 6), stream=stream)
        if record is not None:
            record.append(n_out)
        return n_out

    # error against FP64 and XEB of the samples: the stored oracle amplitudes of call 0
    rel_l2, xeb = None, None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_seed0_call0.npy")
    n_out0 = step(0)
    torch.cuda.synchronize()
    partial_report = None
    if os.path.exists(gold) and args.target_fidelity:
        # psi_X / sqrt(F) is another state: report F against the exact XEB of the
        # batch (the expected XEB of samples drawn from it, Table II's check)
        ref = np.load(gold)
        a = out.cpu().numpy()[0]
        q = a[:, 0].astype(np.float64) ** 2 + a[:, 1].astype(np.float64) ** 2
        p = np.abs(ref) ** 2
        S, X, R = rqc.plan_partial(plan)
        partial_report = {"F": info["fidelity"], "k": len(S), "X": len(X), "sum_R": float(np.sum(R)),
                          "xeb_exact_batch": float((2.0 ** n) * (q * p).sum() / q.sum() - 1.0),
                          "slices": info["n_slices"], "of_total": 1 << info["n_sliced"]}
    elif os.path.exists(gold):
        ref = np.load(gold)
        a = out.cpu().numpy()[0]
        got = a[:, 0].astype(np.float64) + 1j * a[:, 1]
        rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        s = samples.cpu().numpy()[:n_out0].astype(np.uint64)
        t_idx = np.zeros(len(s), dtype=np.int64)
        for b, q in enumerate(open_q):
            t_idx |= ((s >> np.uint64(q)) & np.uint64(1)).astype(np.int64) << b
        if len(s):
            p_exact = np.abs(ref[t_idx]) ** 2
            xeb = {"value": float((2.0 ** n) * p_exact.mean() - 1.0), "samples": int(len(s)),
                   "note": "samples of call 0 scored with the oracle's FP64 probabilities"}
    for w in range(args.warmup):
        step(1 + w)
    torch.cuda.synchronize()
    rqc.plan_profile_reset(plan)
    lat = []
    accepted = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        step(1 + args.warmup + k, accepted)  # the sampler synchronises the stream
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    prof = rqc.plan_profile(plan)
    tree = tree_digest(rqc, plan)
    amps_s = args.steps * (1 << o) / elapsed
    line = {
        "metric": METRIC, "value": amps_s, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * elapsed / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[args.precision], "data": "synthetic",
        "tflops": args.steps * info["flops_per_batch"] / elapsed / 1e12,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "rel_l2_vs_fp64": rel_l2, "xeb_call0": xeb, "partial": partial_report,
        "samples_per_step": float(np.mean(accepted)) if accepted else 0.0,
        "config": {"workload": f"{args.config}: {cfg['rows']}x{cfg['cols']} grid, {cfg['cycles']} cycles, "
                               f"{info['n_slices']} slices ({info['n_sliced']} sliced legs), 2^{o} open batch, "
                               f"alpha {alpha}", "qubits": n, "slices": info["n_slices"], "open_batch": 1 << o,
                   "flops_per_step": info["flops_per_batch"], "gemm_flop_share": info["gemm_flop_share"],
                   "max_log2_tensor": info["max_log2_tensor"], "plan_seconds": plan_s,
                   "launches_per_group": info["n_launches"], "fused_stream_pairs": info["n_fused"],
                   "tree_sha256": tree, "kernel_seconds": {k: v["seconds"] for k, v in prof.items()}},
        "roofline": kernel_roofline(prof, prec == rqc.C64, traffic_key(args, tree)),
    }
    if args.global_cache and not args.target_fidelity:
        # the paper's multi-batch reuse: parts of the contraction that do not
        # depend on the fixed bits are computed once per slice group (the fill)
        # and every batch then contracts only the rest.  Reported beside the
        # headline value, which recomputes everything on every step.
        cplan = rqc.plan_create(circ, open_q, n_sliced_target=n_sliced, path_trials=args.path_trials,
                                path_seed=args.path_seed, precision=prec, global_cache=1, autotune=args.autotune)
        cinfo = rqc.plan_info(cplan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        step(0, pl=cplan)  # fills the cache; call 0 has stored oracle amplitudes
        torch.cuda.synchronize()
        fill_s = time.perf_counter() - t0
        c_rel = None
        if os.path.exists(gold):
            a = out.cpu().numpy()[0]
            ref = np.load(gold)
            c_rel = float(np.linalg.norm(a[:, 0].astype(np.float64) + 1j * a[:, 1] - ref) / np.linalg.norm(ref))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(args.steps):
            step(1 + args.warmup + k, pl=cplan)
        torch.cuda.synchronize()
        c_el = time.perf_counter() - t0
        line["global_cache"] = {
            "ms_per_step": 1e3 * c_el / args.steps, "amplitudes_per_s": args.steps * (1 << o) / c_el,
            "fill_and_first_step_ms": 1e3 * fill_s, "cache_gib": cinfo["cache_bytes"] / 2 ** 30,
            "flops_cached_share": cinfo["flops_cached"] / cinfo["flops_per_batch"],
            "tflops_per_step_executed": args.steps * (cinfo["flops_per_batch"] - cinfo["flops_cached"]) / c_el / 1e12,
            "rel_l2_vs_fp64": c_rel,
            "note": "same steps on a plan whose fixed-bit-independent parts are computed once per slice group "
                    "(filled on the first call, not in this timing; the planner picks the tree by per-batch "
                    "cost), amortised over many batches of one circuit"}
        del cplan
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, text)
    return line


def run_large(args, rqc, torch):
    """One GPU's share of the 53-qubit contraction: slices chosen so that no
    intermediate exceeds 2^30 elements, a share of 2^10 of them; a prefix of
    the slice list is timed and the share, and the 3125 calls that 1e5 samples
    need, are extrapolated linearly (labelled as such)."""
    torch.cuda.set_device(0)
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    o = len(open_q)
    circ = rqc.load_circuit(text)
    t0 = time.perf_counter()
    # full slicing to a 2^30-element memory bound; the share is the first 2^10
    # slices of the slice list.  Partial slicing is not used here: on this
    # path its norm network (the doubled circuit) costs far more than the share
    plan = rqc.plan_create(circ, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                           path_trials=args.path_trials, profile=1)
    plan_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    ids = rqc.plan_slices(plan, cap=args.large_prefix)
    out = torch.empty((1, 1 << o, 2), dtype=torch.float32, device="cuda")
    fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    rqc.contract_amplitudes(plan, fb, out, slice_ids=ids)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t1
    prof = rqc.plan_profile(plan)
    share = 1 << 10
    per_slice = dt / len(ids)
    t_share = per_slice * share
    calls = int(np.ceil(2 * 1e5 / (1 << (o - 6))))
    flops_per_slice = info["flops_per_batch"] / info["n_slices"]
    return {"metric": METRIC, "workload": "large: 6x9 grid minus (0,4), 53 qubits, 20 cycles, one GPU's share "
                                          "of 2^10 slices of a 2^30-element-bounded sliced contraction",
            "plan_seconds": plan_s, "n_sliced": info["n_sliced"], "total_slices": info["n_slices"],
            "flops_per_slice": flops_per_slice, "max_log2_tensor": info["max_log2_tensor"],
            "prefix_slices": len(ids), "prefix_seconds": dt,
            "tflops": flops_per_slice * len(ids) / dt / 1e12,
            "extrapolated_seconds_per_share": t_share,
            "extrapolated_seconds_1e5_samples_at_share": t_share * calls, "calls_for_1e5_samples": calls,
            "label": "measured on a prefix of the slice list, extrapolated linearly (labelled)",
            "kernel_seconds": {k: v["seconds"] for k, v in prof.items()},
            "roofline": kernel_roofline(prof, True)}


def run_serve(args, torch):
    from paper_2112_15083_amd import serve
    torch.cuda.set_device(0)
    kw = dict(shapes=((4, 5), (4, 6), (5, 5), (5, 6)), cycles=(8, 12), log2_amps=(6, 12), samples=(100, 400))
    reqs = serve.synthetic_requests(args.serve_requests, seed=0, rate=None, **kw)
    # capacity: everything submitted at once
    srv = serve.Server(n_streams=4, plan_workers=8)
    t0 = time.perf_counter()
    res = [f.result() for f in [srv.submit(r) for _, r in reqs]]
    cap_s = time.perf_counter() - t0
    srv.shutdown()
    ok = [r for r in res if r.status == "ok"]
    max_rate = len(ok) / cap_s
    loads = {}
    for load in (0.5, 0.8, 1.0):
        rate = load * max_rate
        reqs = serve.synthetic_requests(args.serve_requests, seed=1, rate=rate, **kw)
        srv = serve.Server(n_streams=4, plan_workers=8)
        t0 = time.perf_counter()
        futs = []
        for t, r in reqs:
            while time.perf_counter() - t0 < t:
                time.sleep(0.0005)
            r.arrival = time.perf_counter()
            futs.append(srv.submit(r))
        res = [f.result() for f in futs]
        wall = time.perf_counter() - t0
        srv.shutdown()
        ok = [r for r in res if r.status == "ok"]
        lat = [r.latency for r in ok]
        amps = sum(r.amps.size for r in ok)
        loads[str(load)] = {"offered_rps": rate, "served_rps": len(ok) / wall,
                            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                            "amplitudes_per_s": amps / wall,
                            "tflops": sum(r.flops for r in ok) / wall / 1e12,
                            "refused": sum(r.status == "refused" for r in res),
                            "errors": sum(r.status == "error" for r in res)}
    return {"metric": METRIC, "workload": f"serving: {args.serve_requests} seeded requests per load, "
            "4x5..5x6 grids, 8..14 cycles, 2^6..2^12 amplitudes, half with 1e3..4e3 samples, "
            "half bf16x3", "capacity_rps": max_rate, "loads": loads}


def copy_calibration(torch):
    torch.cuda.set_device(0)
    n = 1 << 27  # 2^27 complex64 = 1 GiB
    x = torch.ones(2 * n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    return {"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="mid", choices=["tiny", "mid", "precision", "large"])
    ap.add_argument("--precision", default="c64", choices=["c64", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path-trials", type=int, default=None,
                    help="randomised greedy trials of the tree search (default 65536; 4096 for large, 256 for tiny)")
    ap.add_argument("--path-seed", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=4,
                    help="time this many of the best estimated trees on the GPU and keep the fastest")
    ap.add_argument("--large-prefix", type=int, default=16)
    ap.add_argument("--target-fidelity", type=float, default=0.0)
    ap.add_argument("--partial-sliced", type=int, default=12)
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=60)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-global-cache", dest="global_cache", action="store_false",
                    help="skip the global-cache measurement reported beside the headline value")
    args = ap.parse_args()
    if args.path_trials is None:
        args.path_trials = {"tiny": 256, "large": 4096}.get(args.config, 65536)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sliced contraction would shard "
              "by slice range across GPUs, which this build does not run.", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        print(json.dumps(copy_calibration(torch)), flush=True)
        return
    if args.serve:
        print(json.dumps(run_serve(args, torch)), flush=True)
        return
    from paper_2112_15083_amd import rqc
    if args.config == "large":
        print(json.dumps(run_large(args, rqc, torch)), flush=True)
        return
    print(json.dumps(run_mid_like(args, rqc, torch)), flush=True)


if __name__ == "__main__":
    main()
