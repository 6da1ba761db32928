"""CPU pins of the partial-slicing oracle (Sec. I.A-I.C, Appendix B)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import circuit as oc
from oracle import partial, stats
from oracle import sv as osv

TEXT = synthetic.circuit_text(4, 4, 10, 0)
CIRC = oc.parse(TEXT)


def _candidates():
    """Variables created by single-qubit gates of cycles 2..5 (a plausible sliced set I)."""
    out = []
    gi_cycle = []
    cyc = 0
    for line in TEXT.splitlines():
        w = line.split()
        if w and w[0] in ("sx", "sy", "sw", "fsim"):
            gi_cycle.append(int(w[1]))
    for (v, g, q) in CIRC.variables():
        if g >= 0 and 2 <= gi_cycle[g] <= 5:
            out.append(v)
    return out


def test_sliced_vertex_select_gives_antichain_of_requested_size():
    I = _candidates()
    S = partial.sliced_vertex_select(CIRC, I, 8)
    assert len(S) == 8 and set(S) <= set(I)
    assert partial.is_antichain(CIRC, S)
    # the first pick has the smallest light cone among all candidates
    lc = partial.LightCones(CIRC)
    sizes = {u: len(lc.vertices([u])) for u in I}
    assert min(len(lc.vertices([v])) for v in S) == min(sizes.values())


def test_light_cone_is_causal_past():
    """L'_C(v) of a first-layer output is just its input variable."""
    lc = partial.LightCones(CIRC)
    first = [v for (v, g, q) in CIRC.variables() if 0 <= g < CIRC.n]
    for v in first[:4]:
        assert lc.vertices([v]) == {lc.gate_inputs[lc.creator[v]][0]}


def test_orthogonality_norms_and_selection():
    I = _candidates()
    S = partial.sliced_vertex_select(CIRC, I, 6)
    psis = [partial.psi_i(TEXT, S, i) for i in range(1 << len(S))]
    G = np.array([[np.vdot(a, b) for b in psis] for a in psis])
    R = np.real(np.diag(G))
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() <= 1e-13                      # <psi_i|psi_i'> = 0
    assert abs(R.sum() - 1.0) <= 1e-12                      # sum_i ||psi_i||^2 = 1
    for f in (0.05, 0.2, 0.5):
        X, F = partial.select_slices(R, f)
        k = len(S)
        assert F >= f
        assert F >= len(X) / 2 ** k - 1e-15                 # Eq. (2)
        assert len(X) <= math.ceil(f * 2 ** k)               # size bound of Sec. I.B
        px = partial.psi_X(TEXT, S, X)
        assert abs(np.vdot(px, px).real - F) <= 1e-12        # ||psi_X||^2 = F
        # minimality: dropping the last chosen index falls below f
        assert F - R[X[-1]] < f


def test_full_alg1_and_xeb_tracks_fidelity():
    """XEB of the normalised partial state against the exact one is about F
    (the Table II relation, here exactly computed instead of sampled)."""
    I = _candidates()
    f = 0.05
    S, R, X, F = partial.slice_selection(TEXT, I, f)
    assert len(S) == math.ceil(3 - math.log2(f))
    p = np.abs(osv.simulate(TEXT)) ** 2
    px = partial.psi_X(TEXT, S, X)
    q = np.abs(px) ** 2 / F
    xeb_exact = (1 << CIRC.n) * float((q * p).sum()) - 1
    assert abs(xeb_exact - F) < 0.5 * F
    # and by sampling 2*10^5 bitstrings from q
    rng = np.random.default_rng(0)
    s = rng.choice(q.size, size=200_000, p=q / q.sum())
    x = stats.xeb(CIRC.n, p[s])
    assert abs(x - xeb_exact) < 4 * math.sqrt(2.0 / s.size) * 3


@pytest.mark.parametrize("rows,cols,cycles,seed,near", [(3, 4, 8, 0, True), (4, 4, 10, 1, True), (3, 4, 8, 2, False)])
def test_lightcone_norms_equal_full_state_vector_norms(rows, cols, cycles, seed, near):
    """Two routes to R: projected full state vectors, and the light cone of S
    split into qubit-disjoint parts.  Near-input S (cones of at most four
    vertices) and a deeper Alg. 2 selection."""
    text = synthetic.circuit_text(rows, cols, cycles, seed)
    c = oc.parse(text)
    lc = partial.LightCones(c)
    n = c.n
    internal = [v for v, gi, q in c.variables() if gi >= 0]
    if near:
        cand = [v for v in internal if len(lc.vertices([v])) <= 4]
        S = []
        for v in cand:
            if all(v not in lc.vertices([u]) and u not in lc.vertices([v]) for u in S):
                S.append(v)
            if len(S) == 6:
                break
    else:
        S = partial.sliced_vertex_select(c, internal[n:n + 40], 5)
    assert partial.is_antichain(c, S)
    a = partial.norms_R(text, S)
    b = partial.norms_R_lightcone(text, S)
    assert abs(a.sum() - 1.0) < 1e-12 and abs(b.sum() - 1.0) < 1e-12
    assert np.abs(a - b).max() <= 1e-13
