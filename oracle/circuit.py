"""ORACLE (test infrastructure): parser of the circuit text and gate matrices.

Gate definitions (the paper uses the grid random circuits of the supremacy
experiment, introduction and Sec. III, without restating them):
  sqrt(P) := (I - iP)/sqrt(2) for P in {X, Y, W}, W = (X + Y)/sqrt(2);
  fSim(theta, phi) in the basis |b_a b_b> (first listed qubit = high bit):
      [[1,0,0,0],[0,cos,-i sin,0],[0,-i sin,cos,0],[0,0,0,exp(-i phi)]].
Variables (tensor legs, Appendix B's vertices): ids 0..n-1 are the qubit
inputs; walking the gate lines in order every single-qubit gate creates one,
fSim with theta = pi/2 creates none (SWAP times a diagonal), any other
two-qubit gate creates two (qa first).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from fractions import Fraction

import numpy as np

X = np.array([[0, 1], [1, 0]], dtype=np.complex128)
Y = np.array([[0, -1j], [1j, 0]], dtype=np.complex128)
W = (X + Y) / np.sqrt(2.0)
PAULI = {"sx": X, "sy": Y, "sw": W}


def one_qubit(name: str) -> np.ndarray:
    return (np.eye(2, dtype=np.complex128) - 1j * PAULI[name]) / np.sqrt(2.0)


def fsim(theta: float, phi: float) -> np.ndarray:
    u = np.zeros((4, 4), dtype=np.complex128)
    u[0, 0] = 1
    u[1, 1] = u[2, 2] = np.cos(theta)
    u[1, 2] = u[2, 1] = -1j * np.sin(theta)
    u[3, 3] = np.exp(-1j * phi)
    return u


@dataclass
class Gate:
    name: str               # sx, sy, sw, fsim
    qubits: tuple
    theta: Fraction = Fraction(0)  # in units of pi
    phi: Fraction = Fraction(0)

    def matrix(self) -> np.ndarray:
        if self.name == "fsim":
            return fsim(np.pi * float(self.theta), np.pi * float(self.phi))
        return one_qubit(self.name)

    @property
    def swap_like(self) -> bool:
        return self.name == "fsim" and self.theta == Fraction(1, 2)


@dataclass
class Circuit:
    n: int
    rows: int = 0
    cols: int = 0
    removed: list = field(default_factory=list)
    cycles: int = 0
    gates: list = field(default_factory=list)

    def variables(self):
        """List of (var_id, gate_index, qubit) for every created variable.

        Input variables have gate_index -1.
        """
        out = [(q, -1, q) for q in range(self.n)]
        nxt = self.n
        for gi, g in enumerate(self.gates):
            if g.name == "fsim":
                if not g.swap_like:
                    out.append((nxt, gi, g.qubits[0])); nxt += 1
                    out.append((nxt, gi, g.qubits[1])); nxt += 1
            else:
                out.append((nxt, gi, g.qubits[0])); nxt += 1
        return out


def parse(text: str) -> Circuit:
    c = Circuit(n=-1)
    for raw in text.splitlines():
        line = raw.split("#", 1)[0].split()
        if not line:
            continue
        w = line[0]
        if w == "qubits":
            c.n = int(line[1])
        elif w == "grid":
            c.rows, c.cols = int(line[1]), int(line[2])
        elif w == "removed":
            c.removed.append((int(line[1]), int(line[2])))
        elif w == "cycles":
            c.cycles = int(line[1])
        elif w in ("sx", "sy", "sw"):
            c.gates.append(Gate(w, (int(line[2]),)))
        elif w == "fsim":
            c.gates.append(Gate("fsim", (int(line[2]), int(line[3])),
                                Fraction(line[4]), Fraction(line[5])))
    if c.n <= 0:
        raise ValueError("circuit text declares no qubits")
    return c
