"""Write searched contraction trees that the tests and the benchmark reuse
(inputs, not expected values).

  mid_tree.json    the 30-qubit "mid" workload's tree (65536 trials, seed 0,
                   its sliced-leg count), on which the tests run the fused
                   streaming pairs;
  large_plan.json  the 53-qubit partial plan's tree and sliced legs from the
                   benchmark's own search (bench.plan_large with its default
                   trials, seeds, annealing moves and selection rule), with
                   the search's parameters and records, so that a run with the
                   same parameters need not repeat a search of a few minutes.

Both are the planner's deterministic results for seeded searches.
Usage:  python tests/data/make_trees.py [mid] [large]
"""
import hashlib
import json
import os
import sys
import types

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from paper_2112_15083_amd import rqc  # noqa: E402

N_SLICED = {"mid": 6}


def large():
    import bench
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    c = rqc.load_circuit(text)
    args = types.SimpleNamespace(path_trials=bench.LARGE_TRIALS, large_seeds=bench.LARGE_SEEDS,
                                 anneal_iters=bench.LARGE_ANNEAL)
    path, legs, records = bench.plan_large(rqc, c, list(cfg["open_qubits"]), args)
    out = {"workload": "large", "circuit_sha256": hashlib.sha256(text.encode()).hexdigest(),
           "search": bench.large_search_params(args), "records": records,
           "path": [list(x) for x in path], "legs": legs}
    with open(os.path.join(HERE, "large_plan.json"), "w") as f:
        json.dump(out, f)


def main():
    which = sys.argv[1:] or ["mid", "large"]
    if "large" in which:
        large()
    if "mid" not in which:
        return
    for name, ns in N_SLICED.items():
        cfg = synthetic.CONFIGS[name]
        text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
        c = rqc.load_circuit(text)
        p = rqc.plan_create(c, cfg["open_qubits"], dry_run=1, n_sliced_target=ns, path_trials=65536, path_seed=0)
        out = {"workload": name, "path_trials": 65536, "path_seed": 0, "n_sliced_target": ns,
               "path": rqc.plan_path(p), "sliced": rqc.plan_sliced_legs(p)}
        with open(os.path.join(HERE, f"{name}_tree.json"), "w") as f:
            json.dump(out, f)


if __name__ == "__main__":
    main()
