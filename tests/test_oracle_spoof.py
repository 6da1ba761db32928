"""CPU pins of the spoofing oracle (Sec. III.B, Appendix A)."""
import itertools
import math

import numpy as np
import pytest

import synthetic
from oracle import circuit as oc
from oracle import partial, spoof, stats
from oracle import sv as osv


def test_batch_size_rule():
    """Step 1: b = ceil(log2(10 N)); the paper's 3M samples take 2^25."""
    assert spoof.batch_size_log2(3_000_000) == 25
    assert spoof.batch_size_log2(1) == 4
    assert spoof.batch_size_log2(1638) == 14 and spoof.batch_size_log2(1639) == 15


def test_select_top_is_the_max_sum_set_with_smallest_indices():
    """Brute force over all subsets of size k: the selection has the largest
    sum of probabilities, and among the sets that do (they differ only in tied
    entries at the threshold) the smallest sum of indices."""
    rng = np.random.default_rng(3)
    for trial in range(40):
        n = int(rng.integers(1, 9))
        p = rng.integers(0, 4, size=n).astype(np.float64) / 4  # many ties
        for k in range(n + 1):
            best = None
            for sub in itertools.combinations(range(n), k):
                key = (-sum(p[list(sub)]), sum(sub))
                if best is None or key < best[0]:
                    best = (key, sub)
            assert list(spoof.select_top(p, k)) == list(best[1]), (p, k)


def test_select_top_order_and_edges():
    p = np.array([0.5, 0.1, 0.5, 0.9, 0.0])
    assert list(spoof.select_top(p, 2)) == [0, 3]          # tie at 0.5: index 0 first
    assert list(spoof.select_top(p, 3)) == [0, 2, 3]       # ascending index order
    assert list(spoof.select_top(p, 0)) == []
    assert list(spoof.select_top(p, 5)) == [0, 1, 2, 3, 4]


def test_probabilities_of_complex64_are_correctly_rounded():
    """(double)re^2 + (double)im^2: both squares are exact in FP64, so the sum is
    the exact rational value rounded once to nearest (fractions), the same
    whether or not the hardware fuses a multiply into the add."""
    from fractions import Fraction
    rng = np.random.default_rng(1)
    a = (rng.standard_normal(200) + 1j * rng.standard_normal(200)).astype(np.complex64)
    p = spoof.probabilities_f32(a)
    for x, px in zip(a, p):
        exact = Fraction(float(x.real)) ** 2 + Fraction(float(x.imag)) ** 2
        assert px == float(exact)  # float(Fraction) rounds to nearest
        assert Fraction(float(x.real)) ** 2 == Fraction(float(x.real) * float(x.real))


def test_expected_top_xeb_matches_monte_carlo_and_eq11():
    """Appendix A at fidelity 1: the exact order-statistic mean against Monte
    Carlo of i.i.d. exponential probabilities, and its large-N limit -ln r."""
    rng = np.random.default_rng(7)
    N = 1024
    for r in (0.1, 0.2, 0.36, 0.5):
        k = int(math.floor(r * N))
        vals = []
        for _ in range(3000):
            x = np.sort(rng.exponential(size=N))[::-1]
            vals.append(x[:k].mean() - 1.0)
        mc, se = float(np.mean(vals)), float(np.std(vals) / math.sqrt(len(vals)))
        assert abs(spoof.expected_top_xeb(N, r) - mc) <= 4 * se, (r, mc, spoof.expected_top_xeb(N, r))
        # Eq. (11): -ln r + O(ln N / N)
        big = spoof.expected_top_xeb(1 << 20, r)
        assert abs(big - (-math.log(r))) <= 20 * math.log(1 << 20) / (1 << 20) + 1e-9
        assert abs(spoof.spoof_xeb_model(1.0, r) + math.log(r)) < 1e-15


def test_partial_fidelity_model_of_appendix_a():
    """Appendix A's model: v = v_f + v_perp with independent uniform parts of
    norms f and 1 - f; keeping the top r N by |v_f|^2 gives XEB -f ln r."""
    rng = np.random.default_rng(11)
    D, f = 1 << 16, 0.3
    vals = {r: [] for r in (0.1, 0.36, 0.5)}
    for _ in range(20):
        vf = (rng.standard_normal(D) + 1j * rng.standard_normal(D)) * math.sqrt(f / (2 * D))
        vp = (rng.standard_normal(D) + 1j * rng.standard_normal(D)) * math.sqrt((1 - f) / (2 * D))
        n_qubits = 16
        for r in vals:
            _, x_s, _ = spoof.spoof_batch(n_qubits, vf, vf + vp, r)
            vals[r].append(x_s)
    for r, v in vals.items():
        # -f ln r plus the finite-N correction of the top order statistics
        want = f * (spoof.expected_top_xeb(D, r) + 1.0) + (1 - f) - 1.0
        assert abs(np.mean(v) - want) <= 4 * np.std(v) / math.sqrt(len(v)) + 1e-3, (r, np.mean(v), want)
        assert abs(want - spoof.spoof_xeb_model(f, r)) < 0.01


@pytest.mark.parametrize("rows,cols,cycles,seed", [(4, 4, 12, 0), (4, 5, 12, 1)])
def test_spoofing_a_circuit_follows_eq12(rows, cols, cycles, seed):
    """The recipe on a real circuit with partial slicing (psi_X of the oracle):
    XEB(S) - XEB(B) is about -F ln r for each r (Eq. (12); Fig. 4's slopes),
    scored with the exact probabilities."""
    text = synthetic.circuit_text(rows, cols, cycles, seed)
    c = oc.parse(text)
    n = c.n
    lc = partial.LightCones(c)
    internal = [v for v, gi, q in c.variables() if gi >= 0]
    # near-input antichain of 6 vertices (Sec. I.B step 1), X by Alg. 1 at f = 0.2
    S = []
    for v in internal:
        if len(lc.vertices([v])) <= 4 and all(v not in lc.vertices([u]) and u not in lc.vertices([v]) for u in S):
            S.append(v)
        if len(S) == 6:
            break
    R = partial.norms_R(text, S)
    X, F = partial.select_slices(R, 0.2)
    approx = partial.psi_X(text, S, X)
    exact = osv.simulate(text)
    # the batch: all 2^n outputs with 4 fixed top qubits (b = n - 4 open qubits)
    open_q = list(range(n - 4))
    fb = synthetic.fixed_bits(n, open_q, 5000 + seed)
    a = osv.batch_amplitudes(approx, fb, open_q)
    e = osv.batch_amplitudes(exact, fb, open_q)
    for r in (0.1, 0.2, 0.36, 0.5):
        keep, x_s, x_b = spoof.spoof_batch(n, a, e, r)
        assert keep.size == int(math.floor(r * a.size))
        # the kept set's exact 2^n p has sd ~ 1.3; tolerance 5 standard errors
        tol = 5 * 1.3 / math.sqrt(keep.size) + 0.02
        assert abs((x_s - x_b) - spoof.spoof_xeb_model(F, r)) <= tol, (r, x_s, x_b, F)
    # and selection by the exact amplitudes (F = 1) gives -ln r
    keep, x_s, x_b = spoof.spoof_batch(n, e, e, 0.36)
    assert abs((x_s - x_b) + math.log(0.36)) <= 0.15
    assert stats.xeb(n, np.abs(e) ** 2) == pytest.approx(x_b)
