"""Write the contraction tree of the 30-qubit "mid" workload that the tests run
the fused streaming pairs on (an input, not an expected value).

Each is the tree the library's planner finds with the benchmark's search
settings (65536 trials, seed 0, the workload's sliced-leg count), stored so
that the tests do not repeat the search.  Usage:  python tests/data/make_trees.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from paper_2112_15083_amd import rqc  # noqa: E402

N_SLICED = {"mid": 6}


def main():
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
