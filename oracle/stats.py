"""ORACLE (test infrastructure): quantities of Secs. II.A-C written from their definitions.

  xeb             linear XEB, Eq. (1): 2^n/k * sum_i p(s_i) - 1
  sampler_law     p'_j = min(p_j, alpha/N_B), eps = sum_j (p_j - p'_j),
                  acceptance per step t = (1 - eps)/alpha,
                  p~_{ij} = p'_j (p_{ij}/p_j) / (1 - eps)          (Sec. II.A)
  tv_distance     D(p, p~) = 1/2 sum |p - p~|                      (Eq. 3)
  fidelity_bound  f' >= f (1 - 4 sqrt(d/f)), valid when d < f/16  (Eq. 9)
  expected_eps    analytic E[eps] under Porter-Thomas (Sec. II.C); the printed
                  formula and the excess-mass reading are both provided
  eps_estimate    empirical estimate from the computed batches J  (Sec. II.C)
"""
from __future__ import annotations

import math

import numpy as np


def xeb(n_qubits: int, probs_of_samples) -> float:
    p = np.asarray(probs_of_samples, dtype=np.float64)
    return float((2.0 ** n_qubits) * p.sum() / p.size - 1.0)


def sampler_law(p: np.ndarray, alpha: float):
    """p: float64 [N_B, N_A], sum 1.  Returns (p_tilde, eps, acceptance)."""
    n_b = p.shape[0]
    p_j = p.sum(axis=1)
    p_prime = np.minimum(p_j, alpha / n_b)
    eps = float((p_j - p_prime).sum())
    ratio = np.divide(p, p_j[:, None], out=np.zeros_like(p), where=p_j[:, None] > 0)
    p_tilde = p_prime[:, None] * ratio / (1.0 - eps)
    return p_tilde, eps, (1.0 - eps) / alpha


def tv_distance(p: np.ndarray, q: np.ndarray) -> float:
    return 0.5 * float(np.abs(np.asarray(p) - np.asarray(q)).sum())


def fidelity_bound(f: float, d: float):
    """Lower bound on the sampled fidelity f' (Eq. 9); None when d >= f/16."""
    if d >= f / 16.0:
        return None
    return f * (1.0 - 4.0 * math.sqrt(d / f))


def expected_eps_printed(n_a: int, n_b: int, alpha: float) -> float:
    """Eq. (10) as printed: N_B * Gamma(N_A, alpha N_A) / Gamma(N_A)."""
    from scipy.special import gammaincc
    return n_b * float(gammaincc(n_a, alpha * n_a))


def expected_eps(n_a: int, alpha: float) -> float:
    """Excess probability mass E[sum_j max(0, p_j - alpha/N_B)] when p_j ~ Gamma(N_A, 2^n).

    For X ~ Gamma(k, rate lam): E[(X - a)+] = (k/lam) Q(k+1, lam a) - a Q(k, lam a);
    with k = N_A, lam a = alpha N_A and N_A N_B = 2^n the sum over N_B batches is
    Q(N_A + 1, alpha N_A) - alpha Q(N_A, alpha N_A).
    """
    from scipy.special import gammaincc
    return float(gammaincc(n_a + 1, alpha * n_a) - alpha * gammaincc(n_a, alpha * n_a))


def eps_estimate(p_j_computed, n_b: int, alpha: float) -> float:
    """N_B * eps_J / |J| with eps_J = sum_{j in J} max(0, p_j - alpha/N_B)."""
    pj = np.asarray(p_j_computed, dtype=np.float64)
    eps_J = float(np.maximum(0.0, pj - alpha / n_b).sum())
    return n_b * eps_J / pj.size
