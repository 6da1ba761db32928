"""ORACLE (test infrastructure): FP64 state vector |psi> = C|0^n> (Sec. I).

Thin ctypes wrapper over sv.c, which is compiled with the system C compiler on
first use (or by the package build step).  For n up to about 30 qubits.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sv.c")
_LIB_PATH = os.path.join(_HERE, "libsvoracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile sv.c into libsvoracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        lib.rqco_num_qubits.argtypes = [ctypes.c_char_p]
        lib.rqco_num_gates.argtypes = [ctypes.c_char_p]
        lib.rqco_simulate.argtypes = [ctypes.c_char_p, ctypes.c_int, ctypes.c_int,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int]
        lib.rqco_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_qubits(text: str) -> int:
    n = _load().rqco_num_qubits(text.encode())
    if n < 0:
        raise ValueError(f"oracle parse error {n}")
    return n


def num_gates(text: str) -> int:
    return _load().rqco_num_gates(text.encode())


def max_threads() -> int:
    return _load().rqco_max_threads()


def simulate(text: str, projections=(), max_gates: int = -1, nthreads: int = 0,
             out: np.ndarray | None = None) -> np.ndarray:
    """Full state vector as complex128[2^n] (index bit q = qubit q).

    projections: iterable of (variable_id, value) projectors (see sv.c).
    max_gates:   simulate only the first gate lines (for timing samples).
    """
    n = num_qubits(text)
    if out is None:
        out = np.empty(1 << n, dtype=np.complex128)
    assert out.dtype == np.complex128 and out.size == (1 << n) and out.flags.c_contiguous
    pv = np.array([p[0] for p in projections] or [0], dtype=np.int32)
    pb = np.array([p[1] for p in projections] or [0], dtype=np.int32)
    rc = _load().rqco_simulate(text.encode(), max_gates, len(projections),
                               pv.ctypes.data, pb.ctypes.data, out.ctypes.data, nthreads)
    if rc != 0:
        raise ValueError(f"oracle simulate error {rc}")
    return out


def batch_indices(fixed_bits: int, open_qubits) -> np.ndarray:
    """Full-state indices of one open batch: entry t has bit open_qubits[b] = bit b of t."""
    o = len(open_qubits)
    t = np.arange(1 << o, dtype=np.int64)
    idx = np.full(1 << o, fixed_bits, dtype=np.int64)
    for b, q in enumerate(open_qubits):
        idx &= ~np.int64(1 << q)
        idx |= ((t >> b) & 1) << q
    return idx


def batch_amplitudes(state: np.ndarray, fixed_bits: int, open_qubits) -> np.ndarray:
    return state[batch_indices(fixed_bits, open_qubits)]
