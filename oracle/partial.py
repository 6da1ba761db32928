"""ORACLE (test infrastructure): partial slicing, Secs. I.A-I.C and Appendix B.

With k partially sliced vertices S on a cut C = C_2 C_1, psi = sum_i psi_i where
psi_i fixes the S-variables to the bits of i (Sec. I.A).  The psi_i are
orthogonal, R[i] = ||psi_i||^2 sums to 1, and keeping a set X of indices gives
psi_X = sum_{i in X} psi_i with fidelity F = sum_{i in X} R[i] (Eq. 2).

psi_i is computed here the plain way: a state-vector run that projects each
S-variable onto its bit right after the gate that creates it (sv.py).

Light cones (Appendix B): L_C(v) is the set of gates v depends on (the causal
past of the gate creating v, itself included); L'_C(v) the set of variables
that are inputs of those gates; for a set, the union over its members.

Bit t of a slice index i is the value of the t-th member of S in ascending
variable-id order.
"""
from __future__ import annotations

import math

import numpy as np

from . import sv as svmod
from .circuit import Circuit, parse


def variable_structure(c: Circuit):
    """Returns (creator, gate_inputs, cone): creator[v] = gate index (-1 for inputs),
    gate_inputs[g] = input variables of gate g, cone[g] = frozenset of gates in
    the causal past of g, g included."""
    cur = list(range(c.n))
    creator = {q: -1 for q in range(c.n)}
    nxt = c.n
    gate_inputs = []
    cone = []
    qcone = [frozenset() for _ in range(c.n)]
    for gi, g in enumerate(c.gates):
        qs = g.qubits
        gate_inputs.append([cur[q] for q in qs])
        cg = frozenset([gi]).union(*[qcone[q] for q in qs])
        cone.append(cg)
        for q in qs:
            qcone[q] = cg
        if g.name == "fsim" and g.swap_like:
            a, b = qs
            cur[a], cur[b] = cur[b], cur[a]
        else:
            for q in qs:
                cur[q] = nxt
                creator[nxt] = gi
                nxt += 1
    return creator, gate_inputs, cone


class LightCones:
    def __init__(self, c: Circuit):
        self.creator, self.gate_inputs, self.cone = variable_structure(c)

    def gates(self, v) -> frozenset:
        g = self.creator[v]
        return frozenset() if g < 0 else self.cone[g]

    def vertices(self, vs) -> set:
        """L'_C of a set of variables."""
        out = set()
        for v in vs:
            for g in self.gates(v):
                out.update(self.gate_inputs[g])
        return out


def sliced_vertex_select(c: Circuit, I, k: int):
    """Appendix B, SlicedVertexSelect(C, I, k), greedy over light-cone size.

    Readings where the printed algorithm is ambiguous: candidates are
    I minus (L'_C(S) union S); the minimised quantity is |L'_C(S u {u})| over
    candidates u; ties go to the smallest variable id.
    """
    lc = LightCones(c)
    S = set()
    while len(S) < k:
        cover = lc.vertices(S)
        cand = sorted(set(I) - cover - S)
        if not cand:
            break
        best = min(cand, key=lambda u: (len(cover | lc.vertices([u])), u))
        S = (S - lc.vertices([best])) | {best}
    return sorted(S)


def is_antichain(c: Circuit, S) -> bool:
    lc = LightCones(c)
    for v in S:
        if lc.vertices([v]) & (set(S) - {v}):
            return False
    return True


def psi_i(text: str, S, i: int, nthreads: int = 0) -> np.ndarray:
    proj = [(v, (i >> t) & 1) for t, v in enumerate(sorted(S))]
    return svmod.simulate(text, projections=proj, nthreads=nthreads)


def norms_R(text: str, S, nthreads: int = 0) -> np.ndarray:
    k = len(S)
    R = np.empty(1 << k, dtype=np.float64)
    for i in range(1 << k):
        v = psi_i(text, S, i, nthreads)
        R[i] = float(np.vdot(v, v).real)
    return R


def norms_R_lightcone(text: str, S) -> np.ndarray:
    """R[i] = ||psi_i||^2 from the light cone C_1 of S alone (Sec. I.A: the gates
    after the cut cancel, ||psi_i||^2 = sum_j |<ji|C_1|0>|^2).  C_1 splits into
    parts that share no qubit; C_1|0> is the tensor product of the parts' states,
    so R is the product of the parts' norm tables.  Each part is a small state
    vector over its own qubits: its gates in circuit order, each S-variable
    projected onto its bit right after the gate that creates it (the
    projection of sv.py).  For S near the inputs this reaches 53-qubit circuits."""
    from . import small
    c = parse(text)
    lc = LightCones(c)
    S = sorted(S)
    k = len(S)
    gates = sorted(set().union(*[lc.gates(v) for v in S])) if S else []
    # qubit carrying each created variable (the gate's qubit for a 1q gate)
    var_qubit = {v: q for v, gi, q in c.variables() if gi >= 0}
    # parts: qubits joined by two-qubit gates of C_1 (union-find)
    parent = {}

    def find(q):
        parent.setdefault(q, q)
        while parent[q] != q:
            parent[q] = parent[parent[q]]
            q = parent[q]
        return q

    for gi in gates:
        qs = c.gates[gi].qubits
        for q in qs:
            find(q)
        if len(qs) == 2:
            parent[find(qs[0])] = find(qs[1])
    parts = {}
    for gi in gates:
        parts.setdefault(find(c.gates[gi].qubits[0]), []).append(gi)
    R = np.ones(1 << k, dtype=np.float64)
    idx = np.arange(1 << k)
    for root, pg in parts.items():
        qubits = sorted({q for gi in pg for q in c.gates[gi].qubits})
        local = {q: t for t, q in enumerate(qubits)}
        mem = [t for t, v in enumerate(S) if lc.creator[v] in set(pg)]
        nq = len(qubits)
        table = np.empty(1 << len(mem))
        for bits in range(1 << len(mem)):
            proj = {lc.creator[S[t]]: (local[var_qubit[S[t]]], (bits >> j) & 1) for j, t in enumerate(mem)}
            psi = np.zeros((2,) * nq, dtype=np.complex128)
            psi[(0,) * nq] = 1.0
            for gi in pg:
                g = c.gates[gi]
                lg = type(g)(g.name, tuple(local[q] for q in g.qubits), g.theta, g.phi)
                psi = small._apply(psi, nq, lg, g.matrix())
                if gi in proj:
                    q, b = proj[gi]
                    sl = [slice(None)] * nq
                    sl[nq - 1 - q] = 1 - b
                    psi[tuple(sl)] = 0.0
            table[bits] = float(np.vdot(psi, psi).real)
        sub_index = np.zeros(1 << k, dtype=np.int64)
        for j, t in enumerate(mem):
            sub_index |= ((idx >> t) & 1) << j
        R *= table[sub_index]
    return R


def select_slices(R: np.ndarray, f: float):
    """Alg. 1's last steps: sort R descending (ties: ascending index), take the
    minimal prefix whose sum reaches f; all of them if rounding never reaches f.
    Returns (X as a list of indices in selection order, F)."""
    order = sorted(range(R.size), key=lambda i: (-R[i], i))
    s = 0.0
    X = []
    for i in order:
        X.append(i)
        s += float(R[i])
        if s >= f:
            break
    return X, float(sum(float(R[i]) for i in X))


def slice_selection(text: str, I, f: float, nthreads: int = 0):
    """Alg. 1 (Appendix B): k0 = ceil(3 - log2 f), S = SlicedVertexSelect(C, I, k0),
    R by the doubled network (here: projected state vectors), X, F."""
    c = parse(text)
    k0 = math.ceil(3 - math.log2(f))
    S = sliced_vertex_select(c, I, k0)
    R = norms_R(text, S, nthreads)
    X, F = select_slices(R, f)
    return S, R, X, F


def psi_X(text: str, S, X, nthreads: int = 0) -> np.ndarray:
    out = None
    for i in X:
        v = psi_i(text, S, i, nthreads)
        out = v.copy() if out is None else out + v
    return out
