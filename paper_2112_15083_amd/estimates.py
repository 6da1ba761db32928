"""Fidelity and sampling-error estimates of Sec. II.B-C (host arithmetic).

  fidelity_bound(F, d)   Eq. (9): the fidelity of the sampled distribution is
                         at least F (1 - 4 sqrt(d / F)) when the sampler's
                         statistical distance d is below F / 16 (None otherwise)
  expected_eps(N_A, a)   Sec. II.C under Porter-Thomas: the batch probability
                         p_j is Gamma(N_A, rate 2^n) and the expected capped
                         mass sum_j E[max(0, p_j - a / N_B)] equals
                         Q(N_A + 1, a N_A) - a Q(N_A, a N_A), Q the regularised
                         upper incomplete gamma function (the printed Eq. (10)
                         counts capped batches instead; see the design notes)
  eps_estimate(p_j, N_B, a)  Sec. II.C empirical estimate N_B eps_J / |J|
"""
from __future__ import annotations

import math


def fidelity_bound(F: float, d: float):
    if not (F > 0) or d >= F / 16.0:
        return None
    return F * (1.0 - 4.0 * math.sqrt(d / F))


def expected_eps(n_a: int, alpha: float) -> float:
    from scipy.special import gammaincc
    return float(gammaincc(n_a + 1, alpha * n_a) - alpha * gammaincc(n_a, alpha * n_a))


def eps_estimate(p_j, n_b: int, alpha: float) -> float:
    total = 0.0
    count = 0
    for p in p_j:
        total += max(0.0, float(p) - alpha / n_b)
        count += 1
    return n_b * total / max(count, 1)
