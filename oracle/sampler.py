"""ORACLE (test infrastructure): the modified frugal rejection sampler of Sec. II.A.

Bitstrings are split b = (b_A, b_B), N_A = 2^|A| (the batch size, 64) and
N_B = 2^(n - |A|).  For a batch j with probabilities p_{i,j}, i in [N_A]:
  1. p_j = sum_i p_{i,j};
  2. accept with probability t_j = min(1, p_j N_B / alpha), alpha > 1;
  3. if accepted, draw i with probability p_{i,j} / p_j.

Exact arithmetic specification (the HIP sampler follows the same one, so the two
give identical samples for identical amplitudes):
  p_{i,j} = (double)re^2 + (double)im^2 from complex64 amplitudes (both products
  exact in FP64); p_j is the sequential FP64 sum over i = 0..N_A-1;
  c = N_B / (alpha * F_norm) in FP64 (F_norm = squared norm of the amplitudes
  handed in, 1 when they are normalised); accept iff U0 < p_j * c;
  i = smallest i whose sequential inclusive prefix sum S_i > U1 * p_j, else the
  last i with p_{i,j} > 0; U_d = Philox uniform with key = seed, draw id d.

Two modes:
  batches   every supplied batch is visited once, in order; the Philox stream
            index of batch j is batch_index_base + j (draw ids 0 and 1);
  pick      (the literal "select j at random" of step 1, for a full vector of
            N_B batches) step t draws j = top log2(N_B) bits of the raw 64-bit
            Philox word (stream t, draw id 2), then uses stream t, ids 0 and 1.
"""
from __future__ import annotations

import numpy as np

from .philox import raw64, uniform53


def probabilities(amps_c64: np.ndarray) -> np.ndarray:
    a = np.asarray(amps_c64, dtype=np.complex64)
    re = a.real.astype(np.float64)
    im = a.imag.astype(np.float64)
    return re * re + im * im


def _sequential_sum(row: np.ndarray) -> float:
    s = 0.0
    for v in row:
        s = s + float(v)
    return s


def _draw_index(row: np.ndarray, p_j: float, u1: float) -> int:
    target = u1 * p_j
    s = 0.0
    last_pos = -1
    for i, v in enumerate(row):
        s = s + float(v)
        if v > 0:
            last_pos = i
        if s > target:
            return i
    return last_pos


def sample_batches(amps: np.ndarray, n_a_log2: int, n_b: int, alpha: float, f_norm: float,
                   seed: int, batch_index_base: int, n_samples: int):
    """Batches mode.  amps: complex64 [n_batches, N_A].

    Returns (list of (batch, i) in ascending batch order, capped at n_samples;
    stats dict).  Pure-Python loops: for small batch counts.
    """
    amps = np.asarray(amps, dtype=np.complex64)
    nb, na = amps.shape
    assert na == 1 << n_a_log2
    p = probabilities(amps)
    c = float(n_b) / (alpha * f_norm)
    u0 = uniform53(seed, np.arange(nb, dtype=np.uint64) + np.uint64(batch_index_base), 0)
    u1 = uniform53(seed, np.arange(nb, dtype=np.uint64) + np.uint64(batch_index_base), 1)
    out = []
    accepted = 0
    used = nb
    eps_j = 0.0
    cap = alpha * f_norm / n_b
    for j in range(nb):
        p_j = _sequential_sum(p[j])
        eps_j += max(0.0, p_j - cap) / f_norm
        if u0[j] < p_j * c:
            accepted += 1
            if len(out) < n_samples:
                out.append((j, _draw_index(p[j], p_j, float(u1[j]))))
                if len(out) == n_samples:
                    used = j + 1
    return out, dict(accepted=accepted, batches=nb, batches_used=used, eps_j=eps_j)


def sample_pick(amps_full: np.ndarray, n_a_log2: int, alpha: float, f_norm: float, seed: int,
                n_samples: int, max_steps: int):
    """Pick mode over a full vector of N_A * N_B amplitudes (index = i + N_A * j)."""
    amps_full = np.asarray(amps_full, dtype=np.complex64)
    na = 1 << n_a_log2
    n_b = amps_full.size // na
    log_nb = n_b.bit_length() - 1
    assert (1 << log_nb) == n_b
    p = probabilities(amps_full).reshape(n_b, na)
    c = float(n_b) / (alpha * f_norm)
    out = []
    steps = 0
    for t in range(max_steps):
        if len(out) == n_samples:
            break
        steps = t + 1
        r = int(raw64(seed, [t], 2)[0])
        j = (r >> (64 - log_nb)) if log_nb > 0 else 0
        p_j = _sequential_sum(p[j])
        u0 = float(uniform53(seed, [t], 0)[0])
        if u0 < p_j * c:
            u1 = float(uniform53(seed, [t], 1)[0])
            out.append((j, _draw_index(p[j], p_j, u1)))
    return out, dict(steps=steps)


def sample_pick_vectorised(p: np.ndarray, alpha: float, seed: int, n_steps: int):
    """Statistical helper: the pick-mode law over many steps at once.

    p: float64 [N_B, N_A] normalised probabilities.  Returns the (j, i) pairs of
    the accepted steps (no cap).  Uses np.cumsum along rows, which adds
    sequentially like the scalar routine above.
    """
    n_b, na = p.shape
    log_nb = n_b.bit_length() - 1
    t = np.arange(n_steps, dtype=np.uint64)
    r = raw64(seed, t, 2)
    j = (r >> np.uint64(64 - log_nb)).astype(np.int64) if log_nb > 0 else np.zeros(n_steps, np.int64)
    cs = np.cumsum(p, axis=1)
    p_j = cs[:, -1]
    u0 = uniform53(seed, t, 0)
    acc = u0 < p_j[j] * (float(n_b) / alpha)
    u1 = uniform53(seed, t, 1)
    ja = j[acc]
    target = u1[acc] * p_j[ja]
    rows = cs[ja]
    i = (rows > target[:, None]).argmax(axis=1)
    return ja, i, int(acc.sum())
