"""Host planning of the 53-qubit partial workload (no GPU): the plan's
partially sliced vertices are the oracle's Alg. 2 selection on the plan's
sliced legs, lie near the inputs (light cones of at most four vertices), form
an antichain, and every intermediate stays within 2^30 elements.  The oracle's
light-cone norms of that S sum to one and give the Table I statistics."""
import math

import numpy as np

import synthetic
from oracle import circuit as oc
from oracle import partial
from paper_2112_15083_amd import rqc

F_TARGET = 2.0 ** -18


def test_large_partial_plan_selects_near_input_antichain():
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    open_q = list(cfg["open_qubits"])
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                        path_trials=1024, path_seed=1, target_fidelity=F_TARGET, dry_run=1)
    info = rqc.plan_info(p)
    legs = rqc.plan_sliced_legs(p)
    S, X, R = rqc.plan_partial(p)
    k0 = math.ceil(3 - math.log2(F_TARGET))
    assert k0 == 21 and len(S) == k0 and info["n_partial"] == k0
    assert X == [] and R == [] and info["fidelity"] == 0.0  # the norms need the GPU
    assert info["max_log2_tensor"] <= 30
    oc_c = oc.parse(text)
    assert S == partial.sliced_vertex_select(oc_c, legs, k0)
    assert partial.is_antichain(oc_c, S)
    lc = partial.LightCones(oc_c)
    assert all(len(lc.vertices([v])) <= 4 for v in S)
    # the same tree and legs with every leg summed stays within the bound
    q = rqc.plan_create(c, open_q, path=rqc.plan_path(p), sliced_legs=legs, max_log2_batched=30, dry_run=1)
    assert rqc.plan_info(q)["max_log2_tensor"] <= 30
    # the oracle's norms of this S (light cone of 53 qubits, split into parts)
    Ro = partial.norms_R_lightcone(text, S)
    assert Ro.size == 1 << 21 and abs(Ro.sum() - 1.0) < 1e-12
    Xo, Fo = partial.select_slices(Ro, F_TARGET)
    assert Fo >= F_TARGET and Fo >= len(Xo) / 2.0 ** k0 and len(Xo) <= math.ceil(F_TARGET * 2 ** k0)


def test_stored_benchmark_plan_follows_its_search():
    """The benchmark's stored 53-qubit plan (tests/data/large_plan.json) is the
    result of the search with the current parameters: regenerate it with
    `python tests/data/make_trees.py large` after changing them.  The kept
    record follows the selection rule, the tree and legs make a valid plan
    within the 2^30-element bound with the recorded estimate, and a search
    with other parameters is not served from the store."""
    import types

    import bench
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    open_q = list(cfg["open_qubits"])
    args = types.SimpleNamespace(path_trials=bench.LARGE_TRIALS, large_seeds=bench.LARGE_SEEDS,
                                 anneal_iters=bench.LARGE_ANNEAL)
    stored = bench.stored_large_plan(text, args)
    assert stored is not None, "stored plan missing or from other search parameters"
    path, legs, recs = stored
    kept = [r for r in recs if r.get("kept")]
    assert len(kept) == 1 and kept[0]["n_sliced"] == len(legs)
    best_job = min(r["est_seconds_all_slices"] for r in recs)
    near = [r for r in recs if r["est_seconds_all_slices"] <= bench.JOB_SLACK * best_job]
    assert kept[0]["est_seconds_share"] == min(r["est_seconds_share"] for r in near)
    c = rqc.load_circuit(text)
    q = rqc.plan_create(c, open_q, path=path, sliced_legs=legs, max_log2_tensor=30, max_log2_batched=30,
                        target_fidelity=bench.LARGE_F, dry_run=1)
    info = rqc.plan_info(q)
    assert info["max_log2_tensor"] <= 30 and info["n_partial"] == 21
    assert abs(info["est_seconds"] - kept[0]["est_seconds_all_slices"]) <= 1e-6 * info["est_seconds"]
    other = types.SimpleNamespace(path_trials=bench.LARGE_TRIALS, large_seeds=bench.LARGE_SEEDS, anneal_iters=1)
    assert bench.stored_large_plan(text, other) is None
