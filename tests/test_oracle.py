"""CPU pins of the oracle: each check compares the oracle with something other
than itself (algebra, an independent route, a closed form, a published value)."""
import math
import os

import numpy as np
import pytest

import synthetic
from oracle import circuit as oc
from oracle import philox, sampler, small, stats
from oracle import sv as osv

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def text(rows, cols, cycles, seed=0, **kw):
    return synthetic.circuit_text(rows, cols, cycles, seed, **kw)


# ---------------------------------------------------------------- generator

def test_generator_deterministic_and_no_repeat():
    a = text(3, 4, 8, seed=3)
    assert a == text(3, 4, 8, seed=3)
    assert a != text(3, 4, 8, seed=4)
    c = oc.parse(a)
    last = {}
    for g in c.gates:
        if g.name != "fsim":
            q = g.qubits[0]
            assert last.get(q) != g.name
            last[q] = g.name


@pytest.mark.parametrize("rows,cols,removed", [(3, 4, ()), (5, 6, ()), (6, 9, ((0, 4),))])
def test_patterns_are_matchings_covering_all_edges(rows, cols, removed):
    sites = synthetic.grid_sites(rows, cols, removed)
    idx = {s: i for i, s in enumerate(sites)}
    edges = set()
    for (r, c) in sites:
        for o in ((r, c + 1), (r + 1, c)):
            if o in idx:
                edges.add(tuple(sorted((idx[(r, c)], idx[o]))))
    seen = set()
    for p in "ABCD":
        pairs = synthetic.pattern_pairs(rows, cols, p, removed)
        qs = [q for pr in pairs for q in pr]
        assert len(qs) == len(set(qs))  # matching
        seen |= set(pairs)
    assert seen == edges


# ---------------------------------------------------------------- gates

def test_gate_unitarity_and_fsim_swap_diag():
    for name in ("sx", "sy", "sw"):
        u = oc.one_qubit(name)
        assert np.abs(u.conj().T @ u - np.eye(2)).max() <= 1e-15
    # sqrt(P)^2 = -iP: the gates are square roots of the Paulis up to phase
    for name, P in oc.PAULI.items():
        u = oc.one_qubit(name)
        assert np.abs(u @ u + 1j * P).max() <= 1e-15
    phi = math.pi / 6
    f = oc.fsim(math.pi / 2, phi)
    assert np.abs(f.conj().T @ f - np.eye(4)).max() <= 1e-15
    swap = np.eye(4)[[0, 2, 1, 3]]
    diag = np.diag([1, -1j, -1j, np.exp(-1j * phi)])
    assert np.abs(f - swap @ diag).max() <= 1e-15


# ---------------------------------------------------------------- state vector

def test_dense_unitary_is_unitary():
    c = oc.parse(text(3, 3, 8, seed=1))
    U = small.dense_unitary(c)
    assert np.abs(U.conj().T @ U - np.eye(U.shape[0])).max() <= 1e-12


def test_c_state_vector_matches_numpy_route_and_norm():
    t = text(3, 4, 8, seed=0)
    a = osv.simulate(t)
    assert abs(np.vdot(a, a).real - 1.0) <= 1e-12
    b = small.numpy_state(oc.parse(t))
    assert np.abs(a - b).max() <= 1e-13


def test_forward_equals_backward_amplitude():
    t = text(3, 4, 10, seed=2)
    a = osv.simulate(t)
    c = oc.parse(t)
    rng = np.random.default_rng(0)
    for x in rng.integers(0, 1 << 12, size=6):
        assert abs(a[x] - small.backward_amplitude(c, int(x))) <= 1e-13


@pytest.mark.parametrize("rows,cols,cycles,seed", [(2, 2, 3, 0), (2, 2, 3, 5), (1, 3, 4, 1)])
def test_path_sum_equals_state_vector(rows, cols, cycles, seed):
    t = text(rows, cols, cycles, seed=seed)
    assert np.abs(small.path_sum(oc.parse(t)) - osv.simulate(t)).max() <= 1e-14


def test_general_fsim_angle_path_sum():
    t = text(2, 2, 3, seed=4, theta="1/3", phi="1/5")
    assert np.abs(small.path_sum(oc.parse(t)) - osv.simulate(t)).max() <= 1e-14


def test_projections_resolve_identity():
    """sum over all values of any set of variables of the projected states = psi."""
    t = text(3, 3, 6, seed=3)
    c = oc.parse(t)
    vids = [v for (v, g, q) in c.variables() if g >= 0]
    rng = np.random.default_rng(1)
    S = sorted(rng.choice(vids, size=4, replace=False).tolist())
    total = sum(osv.simulate(t, projections=[(v, (i >> b) & 1) for b, v in enumerate(S)])
                for i in range(16))
    assert np.abs(total - osv.simulate(t)).max() <= 1e-13


def test_porter_thomas_statistics():
    """2^n p ~ Exp(1) for deep enough random circuits (Sec. II.C, Fig. 2)."""
    ks = []
    xebs = []
    for seed in range(10):
        a = osv.simulate(text(3, 4, 12, seed=seed))
        p = np.abs(a) ** 2
        x = np.sort(p * p.size)
        emp = np.arange(1, x.size + 1) / x.size
        ks.append(np.abs(emp - (1 - np.exp(-x))).max())
        xebs.append(p.size * (p * p).sum() - 1)
    # KS distance of 4096 draws from the true law is ~0.02; 0.06 leaves margin
    assert max(ks) < 0.06
    # exact XEB of ideal sampling, Haar value (2^n - 1)/(2^n + 1) = 0.9995
    assert abs(np.mean(xebs) - 0.9995) < 0.1


# ---------------------------------------------------------------- Philox

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox.philox4x32_10(*v[:6])
        assert [int(o) for o in out] == v[6:]


def test_uniform53_range_and_mean():
    u = philox.uniform53(7, np.arange(200000, dtype=np.uint64), 0)
    assert u.min() >= 0 and u.max() < 1
    assert abs(u.mean() - 0.5) < 0.005


# ---------------------------------------------------------------- sampler

def _full_p(seed=0):
    a = osv.simulate(text(3, 4, 12, seed=seed)).astype(np.complex64)
    p = sampler.probabilities(a)
    return a, p / p.sum()


def test_scalar_and_vectorised_pick_agree():
    """The loop-based sampler and the vectorised helper draw the same samples
    (pins np.cumsum as a sequential sum, as the specification requires)."""
    a, _ = _full_p()
    p = sampler.probabilities(a).reshape(64, 64)
    f_norm = float(p.sum())
    out, st = sampler.sample_pick(a, 6, 2.0, f_norm, 7, 10**9, 3000)
    ja, ia, n_acc = sampler.sample_pick_vectorised(p, 2.0 * f_norm, 7, 3000)
    assert [(int(j), int(i)) for j, i in zip(ja, ia)] == out
    assert n_acc == len(out) > 1000


@pytest.mark.parametrize("alpha", [1.1, 1.2, 2.0])
def test_sampler_output_law_chi2(alpha):
    """Empirical law of 10^6 pick-mode steps vs p~ (Sec. II.A) and acceptance (1-eps)/alpha."""
    _, p = _full_p(seed=1)
    P = p.reshape(64, 64)
    steps = 1_000_000
    ja, ia, n_acc = sampler.sample_pick_vectorised(P, alpha, 11, steps)
    pt, eps, acc = stats.sampler_law(P, alpha)
    # acceptance rate within 5 binomial standard deviations
    sd = math.sqrt(acc * (1 - acc) / steps)
    assert abs(n_acc / steps - acc) < 5 * sd
    # chi^2 over the 64 batch marginals and over all 4096 bitstrings
    cnt_j = np.bincount(ja, minlength=64)
    exp_j = pt.sum(axis=1) * n_acc
    chi_j = float(((cnt_j - exp_j) ** 2 / exp_j).sum())
    assert chi_j < 63 + 6 * math.sqrt(2 * 63)
    cnt = np.bincount(ja * 64 + ia, minlength=4096)
    expc = pt.reshape(-1) * n_acc
    m = expc > 0
    chi = float(((cnt[m] - expc[m]) ** 2 / expc[m]).sum())
    dof = int(m.sum()) - 1
    assert chi < dof + 6 * math.sqrt(2 * dof)
    # D(p, p~) <= eps (Eq. 5)
    assert stats.tv_distance(p, pt.reshape(-1)) <= eps + 1e-15
    if alpha == 1.1:
        assert eps > 1e-3  # capping is exercised


def test_sampler_law_biased_distribution_exercises_caps():
    """A distribution with heavy batches: the closed form still equals the
    empirical law, including for capped batches."""
    rng = np.random.default_rng(5)
    P = rng.exponential(size=(16, 8)) * np.linspace(0.2, 3, 16)[:, None]
    P /= P.sum()
    alpha = 1.5
    pt, eps, acc = stats.sampler_law(P, alpha)
    assert eps > 0.05
    ja, ia, n_acc = sampler.sample_pick_vectorised(P, alpha, 3, 400_000)
    cnt = np.bincount(ja * 8 + ia, minlength=128)
    expc = pt.reshape(-1) * n_acc
    chi = float(((cnt - expc) ** 2 / expc).sum())
    assert chi < 127 + 6 * math.sqrt(2 * 127)
    assert stats.tv_distance(P.reshape(-1), pt.reshape(-1)) <= eps


def test_batches_mode_ordering_and_cap():
    a, _ = _full_p()
    A = a.reshape(64, 64)
    out, st = sampler.sample_batches(A, 6, 64, 2.0, 1.0, 7, 100, 10)
    assert len(out) == min(10, st["accepted"])
    js = [j for j, _ in out]
    assert js == sorted(js) and len(set(js)) == len(js)
    for j, i in out:
        assert abs(A[j, i]) > 0


def test_ideal_samples_xeb_near_one():
    a, p = _full_p(seed=2)
    P = p.reshape(64, 64)
    ja, ia, n = sampler.sample_pick_vectorised(P, 2.0, 5, 40000)
    x = stats.xeb(12, p[ja * 64 + ia])
    assert abs(x - 1.0) < 4 * math.sqrt(2.0 / n)


# ---------------------------------------------------------------- bounds and epsilon

def test_fidelity_bound_worked_example():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "fidelity_bound_example.txt"))
            if l.strip() and not l.startswith("#")]
    f, d, floor = map(float, rows[0])
    b = stats.fidelity_bound(f, d)
    assert b is not None and b >= floor
    assert stats.fidelity_bound(0.01, 0.01 / 16) is None


def test_expected_eps_matches_monte_carlo():
    rng = np.random.default_rng(0)
    for alpha in (1.1, 1.2):
        y = rng.gamma(64, 1 / 64, size=2_000_000)  # p_j N_B under Porter-Thomas
        mc = np.maximum(0, y - alpha).mean()
        assert abs(stats.expected_eps(64, alpha) - mc) < 5e-4 + 0.02 * mc
        # the printed Eq. (10) counts capped batches: N_B * P(p_j N_B > alpha)
        nb = 1 << 20
        assert abs(stats.expected_eps_printed(64, nb, alpha) / nb - (y > alpha).mean()) < 2e-3
    assert stats.expected_eps(64, 2.0) < 1e-10


def test_eps_estimate_unbiased():
    rng = np.random.default_rng(1)
    nb = 4096
    pj = rng.gamma(64, 1 / 64, size=nb) / nb
    full = float(np.maximum(0, pj - 1.1 / nb).sum())
    est = stats.eps_estimate(pj[:2048], nb, 1.1)
    assert abs(est - full) < 0.3 * full + 1e-4


# ---------------------------------------------------------------- Eq. (9) bound: pins from its derivation

def _bures_chain_solution(f, d):
    """The tightest f' that the Bures triangle step of Sec. II.B allows:
    sqrt(1 - sqrt(f')) <= sqrt(1 - sqrt(f)) + sqrt(d), solved for f'."""
    s = 1.0 - (math.sqrt(1.0 - math.sqrt(f)) + math.sqrt(d)) ** 2
    return max(0.0, s) ** 2


def test_fidelity_bound_limits():
    """At the validity edge d = f/16 the factor 1 - 4 sqrt(d/f) is exactly 0,
    and as d -> 0 the bound returns to f.  A bound without the square root
    (0.75 f at the edge) or without the factor 4 (0.75 f as well) fails."""
    for f in (0.002, 0.011, 0.3, 0.9):
        edge = f / 16.0
        b = stats.fidelity_bound(f, edge * (1.0 - 1e-12))
        assert b is not None and 0.0 <= b < 1e-5 * f
        assert stats.fidelity_bound(f, edge) is None
        assert abs(stats.fidelity_bound(f, 1e-40) - f) <= 1e-15 * f
        # half-way in sqrt(d/f): 4 sqrt(d/f) = 1/2 exactly at d = f/64
        assert abs(stats.fidelity_bound(f, f / 64.0) - 0.5 * f) <= 1e-14 * f


def test_fidelity_bound_below_bures_chain():
    """Eq. (9) relaxes the exact solution of the triangle inequality (6)-(8):
    it never exceeds it, and the two agree to first order in sqrt(d) for
    small f (both are f - 4 sqrt(f d) + O(d))."""
    for f in (0.001, 0.01, 0.02, 0.2, 0.7):
        for r in np.linspace(1e-6, 1.0 - 1e-6, 200):
            d = r * f / 16.0
            b = stats.fidelity_bound(f, d)
            assert b is not None and b <= _bures_chain_solution(f, d) + 1e-15
    f, d = 1e-3, 1e-12
    slope_bound = (f - stats.fidelity_bound(f, d)) / math.sqrt(d)
    slope_chain = (f - _bures_chain_solution(f, d)) / math.sqrt(d)
    assert abs(slope_bound / slope_chain * math.sqrt(1.0 - math.sqrt(f)) - 1.0) < 1e-3


def test_fidelity_bound_holds_for_sampled_law():
    """Monte Carlo over random states: psi' with |<psi|psi'>|^2 = f, sampled by
    the Sec. II.A law p~ (alpha chosen to make d small): the classical fidelity
    between |psi|^2 and p~ is at least the bound of Eq. (9) with d = D(p, p~)."""
    rng = np.random.default_rng(11)
    n = 10
    for trial in range(20):
        f = float(rng.uniform(0.05, 0.95))
        psi = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
        psi /= np.linalg.norm(psi)
        perp = rng.normal(size=2 ** n) + 1j * rng.normal(size=2 ** n)
        perp -= np.vdot(psi, perp) * psi
        perp /= np.linalg.norm(perp)
        psi2 = math.sqrt(f) * psi + math.sqrt(1 - f) * perp
        assert abs(abs(np.vdot(psi, psi2)) ** 2 - f) < 1e-12
        p = (np.abs(psi2) ** 2).reshape(16, 64)
        for alpha in (1.05, 1.2, 2.0):
            pt, eps, _ = stats.sampler_law(p, alpha)
            d = stats.tv_distance(p.reshape(-1), pt.reshape(-1))
            assert d <= eps + 1e-15
            b = stats.fidelity_bound(f, d)
            if b is None:
                continue
            q = np.abs(psi) ** 2
            f_cl = float(np.sqrt(q * pt.reshape(-1)).sum() ** 2)
            assert f_cl >= b


# ---------------------------------------------------------------- batches mode: eps_J and the output law

def test_batches_mode_eps_equals_closed_form_with_f_norm():
    """Visiting all N_B batches once, eps_J equals the closed-form eps of
    Sec. II.A, also when the amplitudes are not normalised (F_norm != 1):
    the oracle must divide the capped excess by F_norm."""
    a, p = _full_p(seed=4)
    for scale in (1.0, 0.37, 2.9):
        amps = (a * np.float32(math.sqrt(scale))).astype(np.complex64).reshape(64, 64)
        pr = sampler.probabilities(amps)
        f_norm = float(pr.sum())
        for alpha in (1.1, 1.2, 2.0):
            _, st = sampler.sample_batches(amps, 6, 64, alpha, f_norm, 9, 0, 0)
            _, eps, _ = stats.sampler_law(pr / f_norm, alpha)
            assert abs(st["eps_j"] - eps) <= 1e-12
    # capping is exercised at alpha = 1.1 on this 12-qubit vector
    _, eps11, _ = stats.sampler_law(sampler.probabilities(a.reshape(64, 64)), 1.1)
    assert eps11 > 1e-3


def test_batches_mode_output_law_chi2():
    """Batches mode visits each batch once with its own Philox stream: over
    many visits of 16 batches of N_A = 4, the accepted (j, i) counts follow
    t_j p_ij / p_j, i.e. the closed-form law p~ of Sec. II.A (chi-squared,
    63 degrees of freedom), with heavy batches capped (alpha = 1.2)."""
    rng = np.random.default_rng(6)
    P = rng.exponential(size=(16, 4)) * np.linspace(0.3, 2.5, 16)[:, None]
    P /= P.sum()
    amps = np.sqrt(P).astype(np.complex64)
    pr = sampler.probabilities(amps)
    f_norm = float(pr.sum())
    reps = 6000
    tiled = np.tile(amps, (reps, 1))
    out, st = sampler.sample_batches(tiled, 2, 16, 1.2, f_norm, 21, 12345, 10 ** 9)
    pt, eps, acc_rate = stats.sampler_law(pr / f_norm, 1.2)
    assert eps > 0.05
    cnt = np.zeros(64)
    for j, i in out:
        cnt[(j % 16) * 4 + i] += 1
    n = cnt.sum()
    expc = pt.reshape(-1) * n
    chi = float(((cnt - expc) ** 2 / expc).sum())
    assert chi < 63 + 6 * math.sqrt(2 * 63)
    # acceptance per visited batch: mean of t_j = (1 - eps) / alpha * 16 / N_B (N_B = 16 here)
    rate = st["accepted"] / tiled.shape[0]
    sd = math.sqrt(acc_rate * (1 - acc_rate) / tiled.shape[0])
    assert abs(rate - acc_rate) < 5 * sd


def test_package_estimates_agree_with_oracle():
    """The package's host estimates (used in the benchmark report) against the
    oracle's, which the pins above fix."""
    from paper_2112_15083_amd import estimates
    for f, d in ((0.011, 5e-6), (0.3, 0.001), (2.0 ** -18, 4.3e-12), (0.01, 0.01 / 16)):
        a, b = estimates.fidelity_bound(f, d), stats.fidelity_bound(f, d)
        assert (a is None and b is None) or abs(a - b) <= 1e-15 * f
    for alpha in (1.1, 1.5, 2.0):
        assert abs(estimates.expected_eps(64, alpha) - stats.expected_eps(64, alpha)) <= 1e-15
    rng = np.random.default_rng(2)
    pj = rng.gamma(64, 1 / 64, size=500) / 4096
    assert abs(estimates.eps_estimate(pj, 4096, 1.1) - stats.eps_estimate(pj, 4096, 1.1)) <= 1e-12
