"""Throughput of the sliced-contraction sampler on one MI355X.

One step = one open batch of amplitudes through the whole hot path: leaf
selection per slice group, the contraction program (fused small subtrees,
streaming contractions, permutes, MFMA complex GEMMs), the FP64 cross-slice
sum, normalisation, and rejection sampling over the batch's sub-batches of 64.
Fixed output bits are fresh per step (seeded).  Prints one JSON line.

Default workload ("mid"): 5x6 grid, 14 cycles, 6 sliced legs (64 slices),
2^12-amplitude open batch on the last two rows, alpha = 2.
"""
from __future__ import annotations

import argparse
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
                      f"{amps}-amplitude batch)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="mid", choices=["tiny", "mid", "precision"])
    ap.add_argument("--precision", default="c64", choices=["c64", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path-trials", type=int, default=256)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the sliced contraction shards "
              "by slice range across GPUs, which this build does not run.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2112_15083_amd import rqc

    torch.cuda.set_device(0)
    cfg = synthetic.CONFIGS[args.config]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    o = len(open_q)
    prec = {"c64": rqc.C64, "bf16x3": rqc.BF16X3, "fp16x3": rqc.FP16X3}[args.precision]
    circ = rqc.load_circuit(text)
    t0 = time.perf_counter()
    plan = rqc.plan_create(circ, open_q, n_sliced_target=N_SLICED[args.config], path_trials=args.path_trials,
                           precision=prec, profile=1)
    plan_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    stream = torch.cuda.current_stream()
    out = torch.empty((1, 1 << o, 2), dtype=torch.float32, device="cuda")
    out64 = torch.empty((1, 1 << o, 2), dtype=torch.float64, device="cuda")
    samples = torch.zeros(1 << (o - 6), dtype=torch.int64, device="cuda")
    alpha = cfg["alpha"]

    def step(i, record=None):
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + i)]
        rqc.contract_amplitudes(plan, fb, out, out64, stream=stream)
        n_out, st, _ = rqc.rejection_sample(out, fb, open_q, n, samples.numel(), samples, alpha=alpha,
                                            F_norm=1.0, seed=synthetic.SAMPLER_SEED,
                                            batch_index_base=i << (o - 6), stream=stream)
        if record is not None:
            record.append(n_out)

    # error against FP64: the stored oracle amplitudes of call 0, when present
    rel_l2 = None
    gold = os.path.join(ROOT, "tests", "golden", f"{args.config}_seed0_call0.npy")
    step(0)
    torch.cuda.synchronize()
    if os.path.exists(gold):
        ref = np.load(gold)
        a = out.cpu().numpy()[0]
        got = a[:, 0].astype(np.float64) + 1j * a[:, 1]
        rel_l2 = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
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
    ms = 1e3 * elapsed / args.steps
    amps_s = args.steps * (1 << o) / elapsed
    tflops = args.steps * info["flops_per_batch"] / elapsed / 1e12
    # dominant kernel class by measured time
    cls = max((k for k in prof if k != "sample"), key=lambda k: prof[k]["seconds"])
    pc = prof[cls]
    if cls == "gemm":
        peak = PEAK["fp32_mfma_tflops"] if prec == rqc.C64 else PEAK["bf16_mfma_tflops"]
        achieved = pc["flops"] / pc["seconds"] / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak}
    else:
        achieved = pc["bytes"] / pc["seconds"] / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": achieved / PEAK["hbm_gbs"]}
    roof.update({"kernel": cls, "launches": pc["launches"],
                 "avg_launch_us": 1e6 * pc["seconds"] / max(1, pc["launches"]), "traffic": None})
    line = {
        "metric": METRIC, "value": amps_s, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": {"c64": "complex64 (fp32 MFMA), fp64 slice sum",
                                       "bf16x3": "bf16x3 split (bf16 MFMA), fp64 slice sum",
                                       "fp16x3": "fp16x3 split (fp16 MFMA), fp64 slice sum"}[args.precision],
        "data": "synthetic", "tflops": tflops, "p50_ms": 1e3 * float(np.percentile(lat, 50)),
        "p99_ms": 1e3 * float(np.percentile(lat, 99)), "rel_l2_vs_fp64": rel_l2,
        "samples_per_step": float(np.mean(accepted)) if accepted else 0.0,
        "config": {"workload": f"{args.config}: {cfg['rows']}x{cfg['cols']} grid, {cfg['cycles']} cycles, "
                               f"{info['n_slices']} slices ({info['n_sliced']} sliced legs), 2^{o} open batch, "
                               f"alpha {alpha}", "qubits": n, "slices": info["n_slices"], "open_batch": 1 << o,
                   "flops_per_step": info["flops_per_batch"], "gemm_flop_share": info["gemm_flop_share"],
                   "max_log2_tensor": info["max_log2_tensor"], "plan_seconds": plan_s,
                   "kernel_seconds": {k: v["seconds"] for k, v in prof.items()}},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(cfg, text)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
