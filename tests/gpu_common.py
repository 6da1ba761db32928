"""Helpers shared by the GPU tests: seeded inputs and oracle references."""
import numpy as np

import synthetic
from oracle import sv as osv

# Element-wise bar beside every relative-L2 bar: no entry may be off by more
# than ELEM_FACTOR * tol * rms(ref).  FP32 rounding errors of a contraction are
# close to complex Gaussian with rms = rel-L2 * rms(ref); over 2^14 entries the
# largest is about 3.1 times that rms (P(|e| > k rms) = exp(-k^2)), so a factor
# of 6 never trips on noise at the L2 bar (P < 1e-11) but catches a single wrong
# entry that the norm would average away.
ELEM_FACTOR = 6.0


def circuit(rows, cols, cycles, seed=0, removed=(), **kw):
    return synthetic.circuit_text(rows, cols, cycles, seed, removed, **kw)


def oracle_batches(text, fixed_list, open_qubits, projections=()):
    state = osv.simulate(text, projections=projections)
    return np.stack([osv.batch_amplitudes(state, fb, open_qubits) for fb in fixed_list])


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def max_elem_err(a, b):
    """Largest entry error in units of the reference's rms amplitude."""
    a = np.asarray(a, dtype=np.complex128).ravel()
    b = np.asarray(b, dtype=np.complex128).ravel()
    return float(np.abs(a - b).max() / np.sqrt(np.mean(np.abs(b) ** 2)))


def assert_close(a, b, tol, what=""):
    """rel-L2 <= tol and every entry within ELEM_FACTOR * tol * rms(b)."""
    e2, ei = rel_l2(a, b), max_elem_err(a, b)
    assert e2 <= tol, f"{what}: rel-L2 {e2:.3g} > {tol:.3g}"
    assert ei <= ELEM_FACTOR * tol, f"{what}: entry error {ei:.3g} rms > {ELEM_FACTOR * tol:.3g}"
