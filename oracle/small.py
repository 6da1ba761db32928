"""ORACLE (test infrastructure): independent routes to the amplitudes of tiny circuits.

  numpy_state(c)       state vector by NumPy tensordot, gate by gate
  dense_unitary(c)     the circuit's 2^n x 2^n matrix (columns C|x>)
  backward_amplitude   a(x) = conj(<0| C^dagger |x>), gates undone in reverse
  path_sum(c)          Feynman path sum: one variable per wire segment (every
                       gate gives all its wires a new value), amplitude = sum over
                       all assignments of the product of gate-matrix entries

These pin sv.py: they agree with it only if gate order, qubit/bit convention and
gate matrices are all right.
"""
from __future__ import annotations

import itertools

import numpy as np

from .circuit import Circuit


def _apply(psi: np.ndarray, n: int, gate, u: np.ndarray) -> np.ndarray:
    """psi has shape (2,)*n (+ trailing batch axes); axis n-1-q is qubit q."""
    if len(gate.qubits) == 1:
        ax = n - 1 - gate.qubits[0]
        out = np.tensordot(u, psi, axes=([1], [ax]))
        return np.moveaxis(out, 0, ax)
    qa, qb = gate.qubits
    aa, ab = n - 1 - qa, n - 1 - qb
    u4 = u.reshape(2, 2, 2, 2)  # [a_out, b_out, a_in, b_in]
    out = np.tensordot(u4, psi, axes=([2, 3], [aa, ab]))
    return np.moveaxis(out, [0, 1], [aa, ab])


def numpy_state(c: Circuit, initial: np.ndarray | None = None) -> np.ndarray:
    n = c.n
    if initial is None:
        initial = np.zeros(1 << n, dtype=np.complex128)
        initial[0] = 1
    psi = initial.reshape((2,) * n + initial.shape[1:])
    for g in c.gates:
        psi = _apply(psi, n, g, g.matrix())
    return psi.reshape((1 << n,) + initial.shape[1:])


def dense_unitary(c: Circuit) -> np.ndarray:
    n = c.n
    eye = np.eye(1 << n, dtype=np.complex128)
    return numpy_state(c, eye)


def backward_amplitude(c: Circuit, x: int) -> complex:
    n = c.n
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[x] = 1
    psi = psi.reshape((2,) * n)
    for g in reversed(c.gates):
        psi = _apply(psi, n, g, g.matrix().conj().T)
    return complex(np.conj(psi.reshape(-1)[0]))


def path_sum(c: Circuit) -> np.ndarray:
    """All 2^n amplitudes by explicit enumeration of every wire-segment value."""
    n = c.n
    # wire segment ids: 0..n-1 inputs (fixed to 0), then new ones per gate output
    current = list(range(n))
    nseg = n
    factors = []  # (u, out_ids, in_ids)
    for g in c.gates:
        ins = [current[q] for q in g.qubits]
        outs = []
        for q in g.qubits:
            current[q] = nseg
            outs.append(nseg)
            nseg += 1
        factors.append((g.matrix(), outs, ins))
    free = list(range(n, nseg))  # every non-input segment is summed or is an output
    nfree = len(free)
    if nfree > 24:
        raise ValueError("path sum too large")
    assign = np.arange(1 << nfree, dtype=np.int64)
    val = {s: np.zeros(1 << nfree, dtype=np.int64) for s in range(n)}
    for t, s in enumerate(free):
        val[s] = (assign >> t) & 1
    weight = np.ones(1 << nfree, dtype=np.complex128)
    for u, outs, ins in factors:
        if len(outs) == 1:
            weight = weight * u[val[outs[0]], val[ins[0]]]
        else:
            row = 2 * val[outs[0]] + val[outs[1]]
            col = 2 * val[ins[0]] + val[ins[1]]
            weight = weight * u[row, col]
    x = np.zeros(1 << nfree, dtype=np.int64)
    for q in range(n):
        x |= val[current[q]] << q
    amps = np.zeros(1 << n, dtype=np.complex128)
    np.add.at(amps, x, weight)
    return amps


def all_bitstrings(n: int):
    return itertools.product((0, 1), repeat=n)
