"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This module holds no arithmetic of the method: it only draws random choices and
writes them down as text (circuit files) or integers (fixed output bits).  Both
sides parse the text with their own code and build their own gate matrices.

Circuit family (stand-in for the grid random circuits the paper samples from,
introduction and Sec. III): qubits on a rectangular grid, optionally with sites
removed; each cycle applies one single-qubit gate per qubit drawn from
{sqrt(X), sqrt(Y), sqrt(W)} -- uniform over three at cycle 0, uniform over the
two gates that differ from the qubit's previous gate afterwards -- then
fSim(theta, phi) on the couplers of one of four patterns, cycled ABCDCDAB.

Patterns on the grid (r = row, c = column):
  A: horizontal (r,c)-(r,c+1) with r+c even     B: horizontal with r+c odd
  C: vertical   (r,c)-(r+1,c) with r+c even     D: vertical   with r+c odd
Couplers touching a removed site are dropped.  Qubits are numbered row-major
over the remaining sites.

Text format ("rqc-circuit 1"), one statement per line, '#' starts a comment:
  rqc-circuit 1
  qubits <n>
  grid <rows> <cols>
  removed <r> <c>            (zero or more lines)
  cycles <m>
  sx|sy|sw <cycle> <q>       single-qubit gate on qubit q
  fsim <cycle> <qa> <qb> <t> <p>
                             fSim with theta = pi*t, phi = pi*p, where t and p
                             are written as exact fractions "a/b"
Gate lines are listed in application order.
"""
from __future__ import annotations

import numpy as np

GATE_NAMES = ("sx", "sy", "sw")
PATTERN_ORDER = "ABCDCDAB"


def grid_sites(rows: int, cols: int, removed=()):
    """Row-major list of the (r, c) sites that carry a qubit."""
    rem = {tuple(x) for x in removed}
    return [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in rem]


def pattern_pairs(rows: int, cols: int, pattern: str, removed=()):
    """Couplers of one pattern as (qa, qb) qubit-index pairs, qa < qb."""
    sites = grid_sites(rows, cols, removed)
    index = {s: i for i, s in enumerate(sites)}
    pairs = []
    for (r, c) in sites:
        even = (r + c) % 2 == 0
        if pattern in "AB":
            other = (r, c + 1)
            want_even = pattern == "A"
        else:
            other = (r + 1, c)
            want_even = pattern == "C"
        if even != want_even or other not in index:
            continue
        a, b = index[(r, c)], index[other]
        pairs.append((min(a, b), max(a, b)))
    return sorted(pairs)


def circuit_text(rows: int, cols: int, cycles: int, seed: int, removed=(),
                 theta: str = "1/2", phi: str = "1/6", final_1q_layer: bool = False) -> str:
    """Seeded random grid circuit in the text format above.

    The single-qubit choices come from numpy's PCG64(seed), drawn cycle-major,
    qubit-minor.  With final_1q_layer an extra single-qubit layer (cycle index
    `cycles`) closes the circuit.
    """
    sites = grid_sites(rows, cols, removed)
    n = len(sites)
    rng = np.random.Generator(np.random.PCG64(seed))
    lines = ["rqc-circuit 1", f"qubits {n}", f"grid {rows} {cols}"]
    lines += [f"removed {r} {c}" for (r, c) in removed]
    lines.append(f"cycles {cycles}")
    prev = [-1] * n
    n_layers = cycles + (1 if final_1q_layer else 0)
    for cyc in range(n_layers):
        for q in range(n):
            if prev[q] < 0:
                g = int(rng.integers(0, 3))
            else:
                others = [x for x in range(3) if x != prev[q]]
                g = others[int(rng.integers(0, 2))]
            prev[q] = g
            lines.append(f"{GATE_NAMES[g]} {cyc} {q}")
        if cyc >= cycles:
            break
        pat = PATTERN_ORDER[cyc % len(PATTERN_ORDER)]
        for (a, b) in pattern_pairs(rows, cols, pat, removed):
            lines.append(f"fsim {cyc} {a} {b} {theta} {phi}")
    return "\n".join(lines) + "\n"


def fixed_bits(n_qubits: int, open_qubits, seed: int) -> int:
    """Uniformly random n-bit mask (bit q = qubit q) with the open qubits cleared."""
    rng = np.random.Generator(np.random.PCG64(seed))
    bits = rng.integers(0, 2, size=n_qubits)
    mask = 0
    for q in range(n_qubits):
        if bits[q] and q not in set(open_qubits):
            mask |= 1 << q
    return mask


def fixed_bits_batch(n_qubits: int, open_qubits, first_seed: int, count: int):
    """`count` masks from seeds first_seed, first_seed+1, ..."""
    return [fixed_bits(n_qubits, open_qubits, first_seed + i) for i in range(count)]


# Workloads of the five measured configurations, written as data.
CONFIGS = {
    # 3x4 grid, 8 cycles, no slicing, all 12 qubits open, 1000 samples.
    "tiny": dict(rows=3, cols=4, cycles=8, seed=0, removed=(), n_sliced=0,
                 open_qubits=tuple(range(12)), n_samples=1000, alpha=2.0),
    # 5x6 grid, 14 cycles, 6 sliced legs, open = last two rows (qubits 18..29).
    "mid": dict(rows=5, cols=6, cycles=14, seed=0, removed=(), n_sliced=6,
                open_qubits=tuple(range(18, 30)), alpha=2.0),
    # 5x6 grid, 16 cycles, 10 sliced legs, 2^14 open batch (qubits 16..29).
    "precision": dict(rows=5, cols=6, cycles=16, seed=0, removed=(), n_sliced=10,
                      open_qubits=tuple(range(16, 30)), alpha=2.0),
    # 6x9 grid minus site (0,4): 53 qubits, 20 cycles, 12 open qubits.
    "large": dict(rows=6, cols=9, cycles=20, seed=0, removed=((0, 4),),
                  open_qubits=tuple(range(41, 53)), alpha=2.0),
}

SAMPLER_SEED = 7
FIXED_BITS_SEED = 1000
