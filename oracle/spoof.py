"""ORACLE (test infrastructure): linear-XEB spoofing, Sec. III.B and Appendix A.

The spoofing recipe of Sec. III.B, for N output bitstrings with XEB >= f:
  1. b = ceil(log2(10 N));
  2. a set of b free (open) outputs -- chosen by the caller here;
  3. the amplitudes of the batch B of 2^b bitstrings computed with partial
     slicing at target fidelity f (the projected state psi_X of Sec. I.C);
  4. the N bitstrings of B with the largest |amplitude|.

Written from the definitions:
  batch_size_log2   step 1
  select_top        step 4: the `count` largest probabilities, ties to the
                    smaller batch index, returned in ascending batch index
  spoof_batch       steps 3-4 on a state vector psi_X (partial.py) and the
                    exact state, with the XEB of the kept set and of the batch
  expected_top_xeb  Appendix A for Porter-Thomas (i.i.d. exponential)
                    probabilities at fidelity 1: the exact finite-N mean of the
                    top r N order statistics, E x_(N-j+1) = (1/lambda) sum_{i=j}^N 1/i,
                    whose large-N form is Eq. (11), -ln r
  spoof_xeb_model   Eq. (11) at fidelity f: -f ln r (Appendix A's projection model)
"""
from __future__ import annotations

import math

import numpy as np

from . import stats


def batch_size_log2(n_samples: int) -> int:
    """Sec. III.B step 1: b = ceil(log2(10 N))."""
    return int(math.ceil(math.log2(10 * n_samples)))


def select_top(p, count: int) -> np.ndarray:
    """Indices of the `count` largest entries of p (ties: smaller index first),
    in ascending index order (the definition, by a full stable sort)."""
    p = np.asarray(p)
    count = max(0, min(int(count), p.size))
    order = sorted(range(p.size), key=lambda i: (-p[i], i))
    return np.array(sorted(order[:count]), dtype=np.int64)


def probabilities_f32(amps_c64) -> np.ndarray:
    """|a|^2 of complex64 amplitudes in FP64: (double)re^2 + (double)im^2.  Each
    square is exact (the product of two FP32 values fits an FP64 significand),
    so the sum is rounded once, with or without a fused multiply-add."""
    a = np.asarray(amps_c64, dtype=np.complex64)
    re = a.real.astype(np.float64)
    im = a.imag.astype(np.float64)
    return re * re + im * im


def spoof_batch(n_qubits: int, approx_batch, exact_batch, r: float):
    """Steps 3-4 on one batch: keep the floor(r |B|) entries with the largest
    |approx|^2; returns (kept indices, XEB of the kept set, XEB of the whole
    batch), both XEBs scored with the exact probabilities (Eq. (1))."""
    pa = np.abs(np.asarray(approx_batch)) ** 2
    pe = np.abs(np.asarray(exact_batch)) ** 2
    k = int(math.floor(r * pa.size))
    keep = select_top(pa, k)
    return keep, stats.xeb(n_qubits, pe[keep]), stats.xeb(n_qubits, pe)


def expected_top_xeb(N: int, r: float) -> float:
    """E XEB(S) for S = the top floor(r N) of N i.i.d. Exp(2^n) probabilities
    scored with themselves (Appendix A at f = 1), from the exact order-statistic
    means of the exponential distribution."""
    k = int(math.floor(r * N))
    # E x_(N-j+1) * lambda = H_N - H_{j-1}
    h = np.concatenate([[0.0], np.cumsum(1.0 / np.arange(1, N + 1))])
    top = sum(h[N] - h[j - 1] for j in range(1, k + 1))
    return top / k - 1.0


def spoof_xeb_model(f: float, r: float) -> float:
    """Eq. (11): E XEB(S) = -f ln r (leading order in N)."""
    return -f * math.log(r)
