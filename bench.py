"""Throughput of the sliced-contraction sampler on one MI355X.

Default workload ("large", the 53-qubit share): a 6x9 grid minus site (0,4),
20 cycles, 2^12 open batch, contraction intermediates bounded by 2^30
elements.  Partial slicing (Sec. I.B-I.C, Appendix B) at target fidelity
2^-18 (the kept fraction 2^10 / 2^28 of the workload): 21 partially sliced
vertices near the inputs, their norms R[i] (2^21 entries) contracted on the
GPU from the doubled network, X and F by Alg. 1.  The job is the slice list
X x {0,1}^(|I|-|S|); one GPU's share is 2^10 of its slices (the top-R index
with its first 2^10 completions).  One step = one fixed group of the share's
slices for one fresh batch of fixed bits (contraction, FP64 slice sum,
normalisation by 1/sqrt(F), rejection sampling of the 64 sub-batches); the
share's rate is derived from the steps (the groups have identical shapes) and
labelled as such.

Other workloads (--config):
  mid        5x6 grid, 14 cycles, 6 sliced legs (64 slices), 2^12 batch; one
             step = one batch through the whole path, plus a global-cache run
  precision  5x6 grid, 16 cycles, 10 sliced legs (1024 slices), 2^14 batch,
             in complex64 / bf16x3 / fp16x3 (--precision)
  tiny       3x4 grid, 8 cycles, all 12 qubits open
  spoof      53 qubits, 12 cycles, one 2^25-amplitude batch at fidelity f
             through partial slicing, then the top r of it selected on the GPU
             (linear-XEB spoofing, Sec. III.B)
  verify     the mid circuit: exact amplitudes of sampled bitstrings, 64 per
             step, one batch each with no open qubit, and their FP64 XEB sum
  --serve    the serving loop on a Poisson stream of synthetic requests
  --copy-calibration  a plain 1 GiB device copy, the check of the HBM request
             counters (they read 1 GiB each way for it)

Planning is reported separately (plan_seconds) and is not part of a step.  The
53-qubit plan is the stored result of this benchmark's own seeded search
(tests/data/large_plan.json, written by tests/data/make_trees.py) when the
circuit and every search parameter match; --search repeats the search.
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
EXEC_PEAK_TFLOPS = {0: PEAK["fp32_mfma_tflops"], 1: PEAK["bf16_mfma_tflops"]}


def op_tmin(rec):
    """Binding-roof time of an op's launches: the larger of its executed
    matrix-core (or vector) flops at that unit's peak and its algorithmic
    bytes at the HBM peak."""
    t_flop = rec["exec_flops"] / (EXEC_PEAK_TFLOPS[rec["exec_kind"]] * 1e12)
    t_byte = rec["bytes"] / (PEAK["hbm_gbs"] * 1e9)
    return max(t_flop, t_byte), t_flop, t_byte


def kernel_roofline(op_recs, workload=None):
    """The dominant kernel class by measured time and its place under its
    binding roof.  Per op the binding roof is whichever of the matrix cores
    (executed flops) and HBM (algorithmic bytes) takes longer; `frac` is the
    class's achieved rate over the peak of the roof that binds most of its
    minimum time, and `binding_frac` = sum of per-op minimum times / measured."""
    classes = {}
    for r in op_recs:
        if r["cls"] in ("sample", "select"):
            continue
        c = classes.setdefault(r["cls"], dict(seconds=0.0, flops=0.0, bytes=0.0, exec_flops=0.0, launches=0,
                                              tmin=0.0, t_flop=0.0, t_byte=0.0, kinds=set()))
        tm, tf, tb = op_tmin(r)
        c["seconds"] += r["seconds"]
        c["flops"] += r["flops"]
        c["bytes"] += r["bytes"]
        c["exec_flops"] += r["exec_flops"]
        c["launches"] += r["launches"]
        c["tmin"] += tm
        c["t_flop"] += tf if tf >= tb else 0.0
        c["t_byte"] += tb if tb > tf else 0.0
        if r["exec_flops"] > 0:
            c["kinds"].add(r["exec_kind"])
    cls = max(classes, key=lambda k: classes[k]["seconds"])
    c = classes[cls]
    sec = c["seconds"]
    kind = max(c["kinds"]) if c["kinds"] else 0
    mf = c["exec_flops"] / sec / 1e12
    bw = c["bytes"] / sec / 1e9
    mfma = {"achieved": mf, "peak": EXEC_PEAK_TFLOPS[kind], "unit": "TFLOP/s", "frac": mf / EXEC_PEAK_TFLOPS[kind]}
    hbm = {"achieved": bw, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": bw / PEAK["hbm_gbs"]}
    if c["t_flop"] >= c["t_byte"]:
        roof, other = dict(bound="mfma", **mfma), ("hbm_side", hbm)
    else:
        roof, other = dict(bound="hbm", **hbm), ("mfma_side", mfma)
    roof[other[0]] = other[1]
    roof.update({"binding_frac": c["tmin"] / sec, "kernel": cls, "launches": c["launches"],
                 "avg_launch_us": 1e6 * sec / max(1, c["launches"]),
                 "bytes_per_launch": c["bytes"] / max(1, c["launches"]),
                 "exec_flops_per_launch": c["exec_flops"] / max(1, c["launches"]),
                 "complex_tflops_8_per_mac": c["flops"] / sec / 1e12,
                 "traffic": measured_traffic(cls, workload)})
    return roof


def path_roofline(op_recs, measured_seconds, precision_is_c64=True):
    """Sum over the contraction launches of max(algorithmic flops / matrix-core
    peak, algorithmic bytes / HBM peak), divided by the measured time of the
    same steps.  Algorithmic flops count 8 per complex multiply-add, against the
    FP32 peak (complex64) or the 3-product ceiling of the split GEMMs
    (2516.6 x 8/24 TFLOP/s); permutes, leaf selection, accumulation and the
    sampler have no minimum time of their own and count against the fraction."""
    t = 0.0
    for r in op_recs:
        if r["cls"] not in ("gemm", "stream", "small_trees"):
            continue
        peak = PEAK["fp32_mfma_tflops"]
        if r["cls"] == "gemm" and r["exec_kind"] == 1:
            peak = PEAK["bf16_mfma_tflops"] * 8.0 / 24.0
        t += max(r["flops"] / (peak * 1e12), r["bytes"] / (PEAK["hbm_gbs"] * 1e9))
    return {"tmin_seconds": t, "measured_seconds": measured_seconds, "frac": t / measured_seconds}


def class_seconds(op_recs):
    out = {}
    for r in op_recs:
        out[r["cls"]] = out.get(r["cls"], 0.0) + r["seconds"]
    return out


class SamplerTimer:
    """HIP events around the sampler calls on the stream they run on (the
    sampler entry point synchronises that stream before returning, so the
    second event also covers the host's return from the call).  `cls` names
    the timed class in the per-op records (the top selection uses it too)."""

    def __init__(self, torch, stream, cls="sample"):
        self.torch, self.stream, self.cls = torch, stream, cls
        self.pairs = []

    def __enter__(self):
        self.a = self.torch.cuda.Event(enable_timing=True)
        self.a.record(self.stream)

    def __exit__(self, *exc):
        b = self.torch.cuda.Event(enable_timing=True)
        b.record(self.stream)
        self.pairs.append((self.a, b))

    def reset(self):
        self.pairs = []

    def record(self):
        self.torch.cuda.synchronize()
        sec = sum(a.elapsed_time(b) for a, b in self.pairs) * 1e-3
        return {"cls": self.cls, "op": -1, "launches": len(self.pairs), "seconds": sec, "flops": 0.0,
                "bytes": 0.0, "exec_flops": 0.0, "exec_kind": 0}


# the sources that decide what a given tree executes: the kernels, the
# lowering that picks their tiles and layouts, and the executor (the tree
# search and the planner's estimates are covered by the tree digest instead)
TRAFFIC_SOURCES = ("kernels.hip", "kernels.hpp", "lower.cpp", "runtime.hip")


def source_sha256():
    """One digest over the library sources that decide the traffic of a tree."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_15083_amd", "csrc")
    for name in TRAFFIC_SOURCES:
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

    sampler_time = SamplerTimer(torch, stream)

    def step(i, record=None, pl=None):
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + i)]
        rqc.contract_amplitudes(pl or plan, fb, out, out64, stream=stream)
        with sampler_time:
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
    sampler_time.reset()
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
    op_recs = rqc.plan_profile_ops(plan) + [sampler_time.record()]
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
                   "tree_sha256": tree, "kernel_seconds": class_seconds(op_recs)},
        "roofline": kernel_roofline(op_recs, traffic_key(args, tree)),
        "path_roofline": path_roofline(op_recs, elapsed),
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


LARGE_F = 2.0 ** -18     # target fidelity: the kept fraction 2^10 / 2^28
LARGE_SHARE = 1 << 10    # slices in one GPU's share
LARGE_TRIALS = 4096      # tree-search trials per seed
LARGE_SEEDS = 4          # seeds searched (plan_large states which plan is kept)
LARGE_ANNEAL = 6_000_000 # annealing moves per refined tree, for every seed
JOB_SLACK = 1.5          # plans within this factor of the best estimated job time compete on share time
LARGE_PLAN_FILE = os.path.join(ROOT, "tests", "data", "large_plan.json")


def large_search_params(args):
    return {"path_trials": args.path_trials, "seeds": args.large_seeds, "anneal_iters": args.anneal_iters,
            "job_slack": JOB_SLACK, "target_fidelity": LARGE_F, "max_log2_tensor": 30}


def stored_large_plan(text, args):
    """The stored result of exactly this search (written by
    tests/data/make_trees.py from plan_large), or None: the circuit and every
    search parameter must match."""
    if getattr(args, "search", False) or not os.path.exists(LARGE_PLAN_FILE):
        return None
    rec = json.load(open(LARGE_PLAN_FILE))
    if rec.get("circuit_sha256") != hashlib.sha256(text.encode()).hexdigest() or \
            rec.get("search") != large_search_params(args):
        return None
    return [tuple(x) for x in rec["path"]], rec["legs"], rec["records"]


def plan_large(rqc, circ, open_q, args):
    """Tree and sliced legs for the 53-qubit partial plan: a host-only search per
    seed, each result annealed.  The workload's unit is a share of 2^10 slices,
    so among the plans whose estimated time for the whole job (every slice of
    X x {0,1}^(|I|-k)) is within JOB_SLACK of the best, the one with the
    fastest share (job time / shares per job) is kept: a faster share is never
    bought with a much slower job.  Returns (path, legs, the records of every
    plan considered)."""
    def plan(seed, anneal):
        p = rqc.plan_create(circ, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                            path_trials=args.path_trials, path_seed=seed, target_fidelity=LARGE_F, dry_run=1,
                            anneal_iters=anneal)
        path, legs = rqc.plan_path(p), rqc.plan_sliced_legs(p)
        # a host-only partial plan covers every slice, its S legs looped
        qi = rqc.plan_info(p)
        return path, legs, {"seed": seed, "anneal_iters": anneal, "n_sliced": len(legs),
                            "est_seconds_all_slices": qi["est_seconds"],
                            "est_seconds_share": qi["est_seconds"] * LARGE_SHARE / qi["n_slices"],
                            "flops_per_slice": qi["flops_per_batch"] / qi["n_slices"]}

    results = [plan(seed, 0) for seed in range(args.large_seeds)]
    # simulated annealing of tree and slicing from every seed's search (the
    # best search result does not always anneal to the best plan), the seeds in
    # parallel host threads (the library releases the interpreter while it plans)
    if getattr(args, "anneal_iters", 0) > 0:
        from concurrent.futures import ThreadPoolExecutor
        with ThreadPoolExecutor(max_workers=args.large_seeds) as ex:
            results += list(ex.map(lambda sd: plan(sd, args.anneal_iters), range(args.large_seeds)))
    # the fastest share among the plans near the fastest job; the earlier entry on a tie
    job_best = min(r[2]["est_seconds_all_slices"] for r in results)
    near = [r for r in results if r[2]["est_seconds_all_slices"] <= JOB_SLACK * job_best]
    best = min(near, key=lambda r: r[2]["est_seconds_share"])
    best[2]["kept"] = True
    return best[0], best[1], [r[2] for r in results]


def share_ids(legs, S, x, count, batched):
    """Slice ids of index x of the partially sliced legs S (bit t of x = S[t])
    with the first `count` completions of the other sliced legs.  Completions
    enumerate the batched legs first (so every run of 2^|batched| ids is one
    whole batched group), then the looped legs in ascending slice-id bit."""
    pos = {v: t for t, v in enumerate(legs)}
    base = 0
    for t, v in enumerate(S):
        if (x >> t) & 1:
            base |= 1 << pos[v]
    bset = set(batched)
    rest = sorted(pos[v] for v in batched) + sorted(pos[v] for v in legs if v not in set(S) and v not in bset)
    ids = []
    for c in range(count):
        sid = base
        for j, b in enumerate(rest):
            if (c >> j) & 1:
                sid |= 1 << b
        ids.append(sid)
    return ids


def run_large(args, rqc, torch):
    """One GPU's share of the 53-qubit partial contraction (see the module
    docstring).  Steps time fixed groups of the share's slices; the share's
    rate is derived from them."""
    from paper_2112_15083_amd import estimates
    torch.cuda.set_device(0)
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    o = len(open_q)
    alpha = cfg["alpha"]
    circ = rqc.load_circuit(text)
    t0 = time.perf_counter()
    stored = stored_large_plan(text, args)
    if stored is not None:
        path, legs, tried = stored
        plan_source = "stored result of the same search (tests/data/large_plan.json); --search repeats it"
    else:
        path, legs, tried = plan_large(rqc, circ, open_q, args)
        plan_source = "searched in this run"
    search_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = rqc.plan_create(circ, open_q, path=path, sliced_legs=legs, max_log2_tensor=30, max_log2_batched=30,
                           target_fidelity=LARGE_F, profile=1)
    torch.cuda.synchronize()
    norms_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    S, X, R = rqc.plan_partial(plan)
    R = np.asarray(R)
    k = len(S)
    # the plan's batched legs: legs carried as a tensor mode (slice ids must keep their groups whole)
    group = 1 << info["n_batched"]
    batched = []
    if info["n_batched"]:
        full = rqc.plan_slices(plan, cap=group)
        bits = 0
        for sid in full:
            bits |= sid ^ full[0]
        batched = [v for t, v in enumerate(legs) if (bits >> t) & 1]
    ids = share_ids(legs, S, X[0], LARGE_SHARE, batched)
    G = args.large_group
    assert LARGE_SHARE % G == 0 and G % group == 0
    n_groups = LARGE_SHARE // G
    out = torch.empty((1, 1 << o, 2), dtype=torch.float32, device="cuda")
    samples = torch.zeros(1 << (o - 6), dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    sampler_time = SamplerTimer(torch, stream)
    p_j_seen = []

    def step(i, record=None):
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + i)]
        g = i % n_groups
        rqc.contract_amplitudes(plan, fb, out, slice_ids=ids[g * G:(g + 1) * G], stream=stream)
        with sampler_time:
            n_out, st, _ = rqc.rejection_sample(out, fb, open_q, n, samples.numel(), samples, alpha=alpha,
                                                F_norm=1.0, seed=synthetic.SAMPLER_SEED,
                                                batch_index_base=i << (o - 6), stream=stream)
        if record is not None:
            record.append((n_out, st))

    # the last warm-up step times every class: it names the dominant class, and
    # gives the per-class times and the minimum times of the path roofline (every
    # step runs the same ops on another slice group; the first step also pays
    # the kernels' first launches); the timed steps put events around that
    # class's launches only, the others run back to back
    for w in range(args.warmup):
        if w == args.warmup - 1:
            torch.cuda.synchronize()
            rqc.plan_profile_reset(plan)
        step(w)
    torch.cuda.synchronize()
    warm_recs = rqc.plan_profile_ops(plan) if args.warmup else []
    if warm_recs:
        rqc.plan_profile_classes(plan, [kernel_roofline(warm_recs)["kernel"]])
    rqc.plan_profile_reset(plan)
    sampler_time.reset()
    lat, rec = [], []
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        ts = time.perf_counter()
        step(args.warmup + s_, rec)  # the sampler synchronises the stream
        lat.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    op_recs = rqc.plan_profile_ops(plan) + [sampler_time.record()]
    if warm_recs:
        scale = float(args.steps)
        all_recs = [dict(r, seconds=r["seconds"] * scale, flops=r["flops"] * scale, bytes=r["bytes"] * scale,
                         exec_flops=r["exec_flops"] * scale, launches=r["launches"] * scale) for r in warm_recs]
        kernel_s = dict(class_seconds(all_recs), sample=class_seconds(op_recs).get("sample", 0.0))
        kernel_s_note = (f"per class over the timed steps: the last warm-up step's events x {args.steps} "
                         "(the timed steps time the dominant class only)")
    else:
        all_recs, kernel_s, kernel_s_note = op_recs, class_seconds(op_recs), "from the timed steps"
    flops_per_slice = info["flops_per_batch"] / info["n_slices"] if info["n_slices"] else 0.0
    step_s = elapsed / args.steps
    share_s = step_s * n_groups
    split = large_split_precision(args, rqc, torch, circ, open_q, path, legs, plan, ids, G, n_groups, step_s, n, o,
                                  prof_classes=[kernel_roofline(warm_recs)["kernel"]] if warm_recs else None)
    job_slices = info["n_slices"]
    n_shares = job_slices // LARGE_SHARE
    # fidelity estimate of the job (Sec. II.B-C): F from the norms; eps from the
    # Porter-Thomas expectation at this alpha (the measured eps_J of a group's
    # partial sums is not the job's: its amplitudes are a fraction of psi_X)
    eps_pt = estimates.expected_eps(1 << 6, alpha)
    F = info["fidelity"]
    bound = estimates.fidelity_bound(F, eps_pt)
    calls_1e5 = int(np.ceil(alpha * 1e5 / (1 << (o - 6))))
    line = {
        "metric": METRIC, "value": (1 << o) / share_s, "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE["c64"], "data": "synthetic",
        "value_note": f"2^{o} amplitudes of one share ({LARGE_SHARE} slices) per share time; a step is "
                      f"{G} slices of the share ({n_groups} steps per share, identical shapes): share time = "
                      f"ms_per_step x {n_groups}, derived, not timed as one call",
        "tflops": G * flops_per_slice / step_s / 1e12,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "rel_l2_vs_fp64": None,
        "partial": {
            "target_fidelity": LARGE_F, "k": k, "n_sliced": len(legs), "X": len(X), "F": F,
            "F_lower_bound_eq2": len(X) / 2.0 ** k, "sum_R": float(R.sum()),
            "R_table1": {"sd_normalised": float(np.sqrt((2.0 ** k) * np.var(R * 2.0 ** k) / 2.0 ** k)),
                         "range_normalised": [float(R.min() * 2.0 ** k), float(R.max() * 2.0 ** k)]},
            "norm_network_seconds": norms_s, "job_slices": job_slices, "shares_per_job": n_shares,
            "share": f"index X[0] (top R) with its first {LARGE_SHARE} completions",
            "eps_expected_porter_thomas": eps_pt, "fidelity_bound_eq9": bound,
            "samples_note": "a share's amplitudes are a partial sum of psi_X / sqrt(F); samples of the job need "
                            "all its shares, so the sampler is timed here on the share groups' partial sums "
                            f"(accepted: {sum(r[0] for r in rec)} over {args.steps} steps)",
            "one_gpu_seconds_1e5_samples_extrapolated": share_s * n_shares * calls_1e5,
            "calls_for_1e5_samples": calls_1e5},
        "split_precision": split,
        "config": {"workload": f"large: 6x9 grid minus (0,4), 53 qubits, 20 cycles, 2^{o} open batch, "
                               f"intermediates <= 2^30 elements; partial slicing at f = 2^-18: |I| = {len(legs)} "
                               f"sliced legs, k = {k} near-input partial legs, R on 2^{k} entries, "
                               f"|X| = {len(X)}; one GPU's share = {LARGE_SHARE} of the job's {job_slices} slices; "
                               f"step = {G} slices of the share + sampling of the batch's 64 sub-batches",
                   "qubits": n, "open_batch": 1 << o, "slices_per_step": G, "share_slices": LARGE_SHARE,
                   "flops_per_slice": flops_per_slice, "flops_per_share": flops_per_slice * LARGE_SHARE,
                   "gemm_flop_share": info["gemm_flop_share"], "max_log2_tensor": info["max_log2_tensor"],
                   "plan_seconds": {"tree_search": search_s, "plan_and_norms": norms_s},
                   "plan_source": plan_source,
                   "search": tried, "search_chosen": next(r for r in tried if r.get("kept")),
                   "search_rule": f"fastest estimated share among plans within {JOB_SLACK}x of the fastest "
                                  "estimated job",
                   "launches_per_group": info["n_launches"],
                   "tree_sha256": tree_digest(rqc, plan), "kernel_seconds": kernel_s,
                   "kernel_seconds_note": kernel_s_note,
                   "share_seconds_derived": share_s},
        "roofline": kernel_roofline(op_recs, None),
        "path_roofline": path_roofline(all_recs, elapsed),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_large(text, o, f"the GPU share time is {share_s:.3g} s at F = 2^-18")
    return line


def gate_count(text):
    """Gate lines of a circuit of any width (the oracle's parser; its state
    vector code only takes circuits it can hold)."""
    from oracle import circuit as oc
    return len(oc.parse(text).gates)


def large_split_precision(args, rqc, torch, circ, open_q, path, legs, plan, ids, G, n_groups, step_s, n, o,
                          steps=3, prof_classes=None):
    """The same share steps with the GEMMs in the split modes (fp16x3 with
    power-of-two scaling, bf16x3), timed like the complex64 steps (profiled
    plans, events on the same classes), with each mode's FP64 result on one group of slices compared with
    the complex64 plan's (no FP64 oracle exists at 53 qubits; at 30 qubits the
    modes' errors against the oracle are in the tests)."""
    out = {}
    shape = (1, 1 << o, 2)
    ref64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    amps = torch.empty(shape, dtype=torch.float32, device="cuda")
    fb0 = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED)]
    rqc.contract_amplitudes(plan, fb0, amps, ref64, slice_ids=ids[:G])
    for name, prec in (("fp16x3", rqc.FP16X3), ("bf16x3", rqc.BF16X3)):
        q = rqc.plan_create(circ, open_q, path=path, sliced_legs=legs, max_log2_tensor=30, max_log2_batched=30,
                            target_fidelity=LARGE_F, precision=prec, profile=1)
        if prof_classes:
            rqc.plan_profile_classes(q, prof_classes)
        m64 = torch.empty(shape, dtype=torch.float64, device="cuda")
        rqc.contract_amplitudes(q, fb0, amps, m64, slice_ids=ids[:G])
        torch.cuda.synchronize()
        a = ref64.cpu().numpy()[0]
        b = m64.cpu().numpy()[0]
        rel = float(np.linalg.norm(b - a) / np.linalg.norm(a))
        t0 = time.perf_counter()
        for i in range(steps):
            fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + 100 + i)]
            g = (1 + i) % n_groups
            rqc.contract_amplitudes(q, fb, amps, slice_ids=ids[g * G:(g + 1) * G])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        out[name] = {"ms_per_step": ms, "amplitudes_per_s": (1 << o) / (ms * 1e-3 * n_groups),
                     "speedup_vs_complex64": 1e3 * step_s / ms, "rel_l2_vs_complex64_fp64_sum": rel,
                     "steps": steps}
        del q
    out["note"] = ("contraction only (the complex64 step also samples); relative L2 difference of the FP64 slice "
                   "sums of one group against the complex64 plan")
    return out


def cpu_baseline_large(text, o, gpu_note, budget_s=20.0):
    """The oracle's FP64 state vector on all host cores cannot hold 53 qubits:
    it is timed per gate at 28 qubits over a prefix of this circuit's gate
    list restricted to the first 28 qubits, and extrapolated by 2^25 in state
    size to the 53-qubit circuit (labelled)."""
    from oracle import sv as osv
    lines = text.splitlines()
    keep = []
    n_small = 28
    for ln in lines:
        tok = ln.split()
        if tok and tok[0] == "qubits":
            keep.append(f"qubits {n_small}")
        elif tok and tok[0] in ("sx", "sy", "sw"):
            if int(tok[2]) < n_small:
                keep.append(ln)
        elif tok and tok[0] == "fsim":
            if int(tok[2]) < n_small and int(tok[3]) < n_small:
                keep.append(ln)
        elif tok and tok[0] in ("grid", "removed"):
            continue
        else:
            keep.append(ln)
    small = "\n".join(keep) + "\n"
    n_gates_small = osv.num_gates(small)
    n_gates = gate_count(text)
    threads = osv.max_threads()
    buf = np.empty(1 << n_small, dtype=np.complex128)
    t0 = time.perf_counter()
    osv.simulate(small, max_gates=0, out=buf)
    t_init = time.perf_counter() - t0
    g = 8
    while True:
        t0 = time.perf_counter()
        osv.simulate(small, max_gates=g, out=buf)
        dt = time.perf_counter() - t0 - t_init
        if dt * 2 > budget_s or g >= n_gates_small:
            break
        g = min(n_gates_small, g * 2)
    per_gate_53 = max(dt, 1e-9) / g * 2.0 ** (53 - n_small)
    t_full = per_gate_53 * n_gates
    return {"value": (1 << o) / t_full, "unit": "amplitudes/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 state vector of the first {n_small} qubits over {g} gates ({dt:.1f} s), per-gate time "
                      f"scaled by 2^{53 - n_small} to 53 qubits and by {n_gates} gates (extrapolated, {t_full:.3g} s "
                      f"per 2^{o}-amplitude batch at fidelity 1; {gpu_note})"}


# Linear-XEB spoofing (Sec. III.B, Table IV's first row): 53 qubits, 12 cycles,
# one batch of 2^25 amplitudes at the slicing ratio f = 1.4 %, the top tenth kept
SPOOF = dict(rows=6, cols=9, removed=((0, 4),), cycles=12, seed=0, b=25, f=0.014, r=0.1, trials=4096)


def spoof_open_window(rqc, circ, n, b, trials=128):
    """Sec. III.B step 2: the b free outputs with the least contraction cost,
    searched over windows of b consecutive qubits (the planner's time estimate
    of the full batch, host-only plans)."""
    best = None
    for start in range(0, n - b + 1):
        open_q = list(range(start, start + b))
        p = rqc.plan_create(circ, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                            path_trials=trials, path_seed=0, dry_run=1)
        est = rqc.plan_info(p)["est_seconds"]
        if best is None or est < best[1]:
            best = (open_q, est)
    return best[0]


def run_spoof(args, rqc, torch):
    """One step = the spoofing recipe for one batch: the 2^b amplitudes with
    partial slicing at fidelity f (Sec. I.C, all of X x {0,1}^(|I|-|S|)), then
    the top floor(r 2^b) of them selected on the GPU."""
    torch.cuda.set_device(0)
    cfg = SPOOF
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    circ = rqc.load_circuit(text)
    b = cfg["b"]
    t0 = time.perf_counter()
    open_q = spoof_open_window(rqc, circ, n, b)
    window_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    plan = rqc.plan_create(circ, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                           path_trials=cfg["trials"], path_seed=args.path_seed, target_fidelity=cfg["f"], profile=1)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    S, X, R = rqc.plan_partial(plan)
    count = int(np.floor(cfg["r"] * (1 << b)))
    out = torch.empty((1, 1 << b, 2), dtype=torch.float32, device="cuda")
    sel = torch.empty(count, dtype=torch.int64, device="cuda")
    stream = torch.cuda.current_stream()
    sel_time = SamplerTimer(torch, stream, cls="select")

    def step(i):
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + i)]
        rqc.contract_amplitudes(plan, fb, out, stream=stream)
        with sel_time:
            rqc.select_top(out, fb[0], open_q, n, count, sel, stream=stream)

    for w in range(args.warmup):
        step(w)
    torch.cuda.synchronize()
    rqc.plan_profile_reset(plan)
    sel_time.reset()
    lat = []
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        ts = time.perf_counter()
        step(args.warmup + s_)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - ts)
    elapsed = time.perf_counter() - t_start
    op_recs = rqc.plan_profile_ops(plan) + [sel_time.record()]
    step_s = elapsed / args.steps
    F = info["fidelity"]
    line = {
        "metric": METRIC, "value": (1 << b) / step_s, "unit": "amplitudes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE["c64"], "data": "synthetic",
        "samples_per_s": count / step_s, "tflops": info["flops_per_batch"] / step_s / 1e12,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "spoof": {"b": b, "samples_per_batch": count, "r": count / (1 << b), "target_fidelity": cfg["f"],
                  "F": F, "k": len(S), "X": len(X), "job_slices": info["n_slices"],
                  "expected_xeb_eq11": -F * float(np.log(count / (1 << b))),
                  "select_ms_per_step": 1e3 * op_recs[-1]["seconds"] / max(1, op_recs[-1]["launches"]),
                  "note": "XEB of the kept set expected at -F ln r above the batch's own (Eq. (11)-(12)); "
                          "the relation is checked against exact probabilities on 20-qubit circuits in the tests"},
        "config": {"workload": f"spoof: 6x9 grid minus (0,4), 53 qubits, {cfg['cycles']} cycles; one batch of "
                               f"2^{b} amplitudes on the {b} cheapest consecutive open qubits (from {open_q[0]}), "
                               f"partial slicing at f = {cfg['f']} (k = {len(S)}, |X| = {len(X)}, "
                               f"{info['n_slices']} slices); step = the batch + top-{count} selection",
                   "qubits": n, "open_qubits": open_q, "flops_per_batch": info["flops_per_batch"],
                   "gemm_flop_share": info["gemm_flop_share"], "max_log2_tensor": info["max_log2_tensor"],
                   "plan_seconds": {"open_window_search": window_s, "plan_and_norms": plan_s},
                   "tree_sha256": tree_digest(rqc, plan), "kernel_seconds": class_seconds(op_recs)},
        "roofline": kernel_roofline(op_recs, None),
        "path_roofline": path_roofline(op_recs, elapsed),
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline_large(text, b, f"the GPU batch time is {step_s:.3g} s at F = {F:.3g}")
    return line



# Verification of produced samples (Sec. III.A): the 30-qubit circuit's samples
# get their exact amplitudes one bitstring per batch (no open qubit)
VERIFY_BITS = 64


def run_verify(args, rqc, torch):
    """Samples of the 30-qubit workload, drawn from correlated 2^12 batches,
    are verified with exact amplitudes: each sampled bitstring is a batch of
    its own with no open qubit, on a plan whose bitstring-independent subtrees
    stay in the global cache.  One step = one call over VERIFY_BITS sampled
    bitstrings; the samples' linear XEB follows from the verified
    probabilities."""
    torch.cuda.set_device(0)
    cfg = synthetic.CONFIGS["mid"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    o = len(open_q)
    circ = rqc.load_circuit(text)
    stream = torch.cuda.current_stream()
    # the samples to verify, from the correlated-batch pipeline
    t0 = time.perf_counter()
    splan = rqc.plan_create(circ, open_q, n_sliced_target=N_SLICED["mid"], path_trials=args.path_trials,
                            path_seed=args.path_seed)
    out = torch.empty((1, 1 << o, 2), dtype=torch.float32, device="cuda")
    samples = torch.zeros(1 << (o - 6), dtype=torch.int64, device="cuda")
    n_calls = max(1, args.warmup) + args.steps  # the first call fills the cache
    need = VERIFY_BITS * n_calls
    drawn, seen, call = [], [], 0
    while len(drawn) < need:
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + 500 + call)]
        rqc.contract_amplitudes(splan, fb, out, stream=stream)
        n_out, _, _ = rqc.rejection_sample(out, fb, open_q, n, samples.numel(), samples, alpha=cfg["alpha"],
                                           F_norm=1.0, seed=synthetic.SAMPLER_SEED,
                                           batch_index_base=(call + 4096) << (o - 6), stream=stream)
        a = out.cpu().numpy()[0]
        for s_ in samples.cpu().numpy()[:n_out].astype(np.uint64):
            t = 0
            for j, q in enumerate(open_q):
                t |= int((int(s_) >> q) & 1) << j
            drawn.append(int(s_))
            seen.append(complex(float(a[t, 0]), float(a[t, 1])))
        call += 1
    sample_s = time.perf_counter() - t0
    del splan
    t0 = time.perf_counter()
    plan = rqc.plan_create(circ, [], n_sliced_target=N_SLICED["mid"], path_trials=args.path_trials,
                           path_seed=args.path_seed, global_cache=1, profile=1)
    plan_s = time.perf_counter() - t0
    info = rqc.plan_info(plan)
    vall = torch.empty((n_calls * VERIFY_BITS, 1, 2), dtype=torch.float32, device="cuda")
    part = torch.empty(n_calls, dtype=torch.float64, device="cuda")

    def step(i):
        # exact amplitudes of the step's bitstrings, then their FP64 sum of Eq. (1)
        v = vall[i * VERIFY_BITS:(i + 1) * VERIFY_BITS]
        rqc.contract_amplitudes(plan, drawn[i * VERIFY_BITS:(i + 1) * VERIFY_BITS], v, stream=stream)
        rqc.prob_sums(v, 1, VERIFY_BITS, n, part[i:i + 1], stream=stream)
        stream.synchronize()

    t0 = time.perf_counter()
    step(0)  # fills the cache
    fill_s = time.perf_counter() - t0
    for w in range(1, args.warmup):
        step(w)
    rqc.plan_profile_reset(plan)
    lat = []
    t_start = time.perf_counter()
    for s_ in range(args.steps):
        ts = time.perf_counter()
        step(max(1, args.warmup) + s_)
        lat.append(time.perf_counter() - ts)
    elapsed = time.perf_counter() - t_start
    op_recs = rqc.plan_profile_ops(plan)
    step_s = elapsed / args.steps
    # the samples' XEB (Eq. (1)) over every verified amplitude, on the GPU
    k = n_calls * VERIFY_BITS
    xeb_d = torch.empty(1, dtype=torch.float64, device="cuda")
    sum_d = torch.empty(1, dtype=torch.float64, device="cuda")
    rqc.prob_sums(vall, 1, k, n, sum_d, xeb_d, stream=stream)
    stream.synchronize()
    xeb = float(xeb_d.item())
    v = vall.cpu().numpy()[:, 0, :]
    amps = v[:, 0].astype(np.float64) + 1j * v[:, 1]
    ref = np.array(seen[:k])
    rel = float(np.linalg.norm(amps - ref) / np.linalg.norm(ref))
    xeb_sigma = float(np.std((2.0 ** n) * np.abs(amps) ** 2) / np.sqrt(k))
    step_sums = part.cpu().numpy()
    per_bitstring = info["flops_per_batch"] - info["flops_cached"]
    line = {
        "metric": METRIC, "value": VERIFY_BITS / step_s, "unit": "amplitudes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * step_s, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE["c64"], "data": "synthetic",
        "tflops": VERIFY_BITS * per_bitstring / step_s / 1e12,
        "p50_ms": 1e3 * float(np.percentile(lat, 50)), "p99_ms": 1e3 * float(np.percentile(lat, 99)),
        "verify": {"bitstrings_verified": int(len(amps)), "samples_drawn": len(drawn),
                   "correlated_calls": call, "sampling_seconds": sample_s,
                   "xeb_of_samples": xeb, "xeb_sigma": xeb_sigma,
                   "xeb_from_step_sums": float((2.0 ** n) * step_sums.sum() / k - 1.0),
                   "rel_l2_vs_sampled_batch_amplitudes": rel,
                   "cache_fill_and_first_step_ms": 1e3 * fill_s, "cache_gib": info["cache_bytes"] / 2 ** 30,
                   "flops_cached_share": info["flops_cached"] / info["flops_per_batch"],
                   "note": "the verified amplitudes come from another contraction tree than the batches the "
                           "samples were drawn from; the relative L2 difference compares the two"},
        "config": {"workload": f"verify: the 30-qubit circuit (5x6 grid, {cfg['cycles']} cycles), samples drawn "
                               f"from correlated 2^{o} batches, exact amplitudes of {VERIFY_BITS} sampled "
                               f"bitstrings per step, one per batch with no open qubit, {info['n_slices']} slices, "
                               f"global cache, then the step's FP64 sum of Eq. (1)",
                   "qubits": n, "flops_per_bitstring": per_bitstring, "n_slices": info["n_slices"],
                   "gemm_flop_share": info["gemm_flop_share"], "max_log2_tensor": info["max_log2_tensor"],
                   "plan_seconds": plan_s, "tree_sha256": tree_digest(rqc, plan),
                   "kernel_seconds": class_seconds(op_recs)},
        "roofline": kernel_roofline(op_recs, None),
        "path_roofline": path_roofline(op_recs, elapsed),
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(cfg, text)
        t_sv = (1 << o) / cb["value"]
        cb["value"] = VERIFY_BITS / t_sv
        cb["sample"] += f"; per step's {VERIFY_BITS} bitstrings: {VERIFY_BITS} / {t_sv:.0f} s"
        line["cpu_baseline"] = cb
    return line


# The serving workload: seeded random grid circuits of 20-40 qubits, 8-20
# cycles, 2^6-2^13 amplitudes, half of them also asking for 1e3-1e4 samples,
# half in bf16x3; requests whose plan costs more than SERVE_CAP flops are
# refused and counted
SERVE_KW = dict(shapes=((4, 5), (4, 6), (5, 5), (5, 6), (5, 7), (6, 6), (5, 8)), cycles=(8, 20), log2_amps=(6, 13),
                samples=(1000, 10000), sample_frac=0.5, bf16_frac=0.5, min_log2_for_samples=13)
SERVE_CAP = 2e13


def serve_workload_text(n, kw, cap):
    shapes = ", ".join(f"{r}x{c}" for r, c in kw["shapes"])
    qubits = sorted(r * c for r, c in kw["shapes"])
    return (f"serving: {n} seeded requests per load, grids {shapes} ({qubits[0]}..{qubits[-1]} qubits), "
            f"{kw['cycles'][0]}..{kw['cycles'][1]} cycles, 2^{kw['log2_amps'][0]}..2^{kw['log2_amps'][1]} amplitudes, "
            f"{int(100 * kw['sample_frac'])}% also asking for {kw['samples'][0]}..{kw['samples'][1]} samples "
            f"(in batches of 2^{kw['min_log2_for_samples']}), "
            f"{int(100 * kw['bf16_frac'])}% bf16x3; plan-cost cap {cap:.0e} flops (above it: refused)")


def run_serve(args, torch):
    from paper_2112_15083_amd import serve
    torch.cuda.set_device(0)
    kw = dict(SERVE_KW)
    n = args.serve_requests
    t_all = time.perf_counter()
    reqs = serve.synthetic_requests(n, seed=0, rate=None, **kw)
    # capacity: everything submitted at once
    srv = serve.Server(n_streams=4, plan_workers=16, plan_flops_cap=SERVE_CAP)
    t0 = time.perf_counter()
    res = [f.result() for f in [srv.submit(r) for _, r in reqs]]
    cap_s = time.perf_counter() - t0
    cap_stats = dict(srv.stats)
    srv.shutdown()
    ok = [r for r in res if r.status == "ok"]
    # the loads below offer the same mix (refused requests included), so the
    # capacity is counted over every submitted request
    max_rate = n / cap_s
    print(f"capacity run: {len(ok)} served, {cap_stats['refused']} refused in {cap_s:.1f} s", flush=True)
    loads = {}
    for load in (0.5, 0.8, 1.0):
        rate = load * max_rate
        reqs = serve.synthetic_requests(n, seed=1, rate=rate, **kw)
        srv = serve.Server(n_streams=4, plan_workers=16, plan_flops_cap=SERVE_CAP)
        t0 = time.perf_counter()
        futs = []
        for t, r in reqs:
            while time.perf_counter() - t0 < t:
                time.sleep(0.0005)
            r.arrival = time.perf_counter()
            futs.append(srv.submit(r))
        res = [f.result() for f in futs]
        wall = time.perf_counter() - t0
        st = dict(srv.stats)
        srv.shutdown()
        ok = [r for r in res if r.status == "ok"]
        lat = [r.latency for r in ok]
        amps = sum(r.amps.size for r in ok)
        loads[str(load)] = {"offered_rps": rate, "served_rps": len(ok) / wall,
                            "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                            "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                            "amplitudes_per_s": amps / wall,
                            "samples_per_s": sum(r.n_samples for r in ok) / wall,
                            "tflops": sum(r.flops for r in ok) / wall / 1e12,
                            "served": len(ok), "refused": st["refused"], "short": st["short"],
                            "errors": st["errors"], "work_units": st["units"],
                            "plan_cache_hits": st["plan_cache_hits"], "extra_sampling_rounds": st["extra_rounds"],
                            "qubits_served": [min(r_.n_qubits for _, r_ in reqs), max(r_.n_qubits for _, r_ in reqs)]}
        print(f"load {load}: {len(ok)} served, p50 {loads[str(load)]['p50_ms']:.1f} ms, "
              f"p99 {loads[str(load)]['p99_ms']:.1f} ms", flush=True)
    return {"metric": METRIC, "workload": serve_workload_text(n, kw, SERVE_CAP), "requests_per_load": n,
            "capacity_rps": max_rate, "capacity_served_rps": len(ok) / cap_s,
            "capacity_note": "requests of the mix (refused ones included) per second with all submitted at once; "
                             "each load offers that fraction of it as Poisson arrivals",
            "capacity_run": {"seconds": cap_s, **cap_stats}, "loads": loads,
            "wall_seconds": time.perf_counter() - t_all}


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
    ap.add_argument("--config", default="large", choices=["tiny", "mid", "precision", "large", "spoof", "verify"])
    ap.add_argument("--precision", default="c64", choices=["c64", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--path-trials", type=int, default=None,
                    help="randomised greedy trials of the tree search (default 65536; 4096 for large, 256 for tiny)")
    ap.add_argument("--path-seed", type=int, default=0)
    ap.add_argument("--autotune", type=int, default=4,
                    help="time this many of the best estimated trees on the GPU and keep the fastest")
    ap.add_argument("--large-group", type=int, default=32,
                    help="slices of the 53-qubit share per step (the share is 1024 slices)")
    ap.add_argument("--large-seeds", type=int, default=LARGE_SEEDS,
                    help="tree-search seeds for the 53-qubit plan (see plan_large for which plan is kept)")
    ap.add_argument("--search", action="store_true",
                    help="search the 53-qubit plan even when the stored result of the same search exists")
    ap.add_argument("--anneal-iters", type=int, default=LARGE_ANNEAL,
                    help="simulated-annealing moves per refined tree for the 53-qubit plan (0 = search only)")
    ap.add_argument("--target-fidelity", type=float, default=0.0)
    ap.add_argument("--partial-sliced", type=int, default=12)
    ap.add_argument("--serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true")
    ap.add_argument("--no-global-cache", dest="global_cache", action="store_false",
                    help="skip the global-cache measurement reported beside the headline value")
    args = ap.parse_args()
    if args.path_trials is None:
        args.path_trials = {"tiny": 256, "large": LARGE_TRIALS}.get(args.config, 65536)
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
    if args.config == "spoof":
        print(json.dumps(run_spoof(args, rqc, torch)), flush=True)
        return
    if args.config == "verify":
        print(json.dumps(run_verify(args, rqc, torch)), flush=True)
        return
    print(json.dumps(run_mid_like(args, rqc, torch)), flush=True)


if __name__ == "__main__":
    main()
