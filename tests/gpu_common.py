"""Helpers shared by the GPU tests: seeded inputs and oracle references."""
import numpy as np

import synthetic
from oracle import sv as osv


def circuit(rows, cols, cycles, seed=0, removed=(), **kw):
    return synthetic.circuit_text(rows, cols, cycles, seed, removed, **kw)


def oracle_batches(text, fixed_list, open_qubits, projections=()):
    state = osv.simulate(text, projections=projections)
    return np.stack([osv.batch_amplitudes(state, fb, open_qubits) for fb in fixed_list])


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
