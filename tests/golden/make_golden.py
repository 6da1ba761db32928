"""Write the stored FP64 expected amplitudes for the 30-qubit workloads.

Calls only the oracle (full 2^30 state vector, 16 GiB of host memory) and the
seeded input generator.  Usage:  python tests/golden/make_golden.py [mid|precision ...]
Each output file holds complex128 amplitudes of one open batch, in the batch's
own index order (bit b of the index = open_qubits[b]).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synthetic  # noqa: E402
from oracle import sv as osv  # noqa: E402

N_CALLS = 2  # fixed-bit seeds FIXED_BITS_SEED + 0, + 1


def golden_path(name: str, call: int) -> str:
    return os.path.join(HERE, f"{name}_seed0_call{call}.npy")


def make(name: str, nthreads: int = 0):
    cfg = synthetic.CONFIGS[name]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = osv.num_qubits(text)
    t0 = time.time()
    state = osv.simulate(text, nthreads=nthreads)
    dt = time.time() - t0
    print(f"{name}: {n} qubits simulated in {dt:.1f} s", flush=True)
    for call in range(N_CALLS):
        fb = synthetic.fixed_bits(n, cfg["open_qubits"], synthetic.FIXED_BITS_SEED + call)
        amps = osv.batch_amplitudes(state, fb, cfg["open_qubits"])
        np.save(golden_path(name, call), amps.astype(np.complex128))
    with open(os.path.join(HERE, f"{name}_seed0_timing.txt"), "w") as f:
        f.write(f"# oracle full state vector, {n} qubits, {osv.max_threads() if nthreads <= 0 else nthreads}"
                f" threads: {dt:.1f} s\n")


if __name__ == "__main__":
    names = sys.argv[1:] or ["mid", "precision"]
    for nm in names:
        make(nm)
