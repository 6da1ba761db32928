"""ORACLE -- test infrastructure, not part of the product.

A plain, slow, obviously correct CPU implementation of what the sampler's hot
path computes, written from the paper (arXiv 2112.15083) and sharing no code
with the HIP library:

  circuit.py   own parser of the circuit text and the gate matrices
  sv.py        FP64 state vector |psi> = C|0> (C/OpenMP in sv.c; Sec. I)
  small.py     NumPy state vector, dense unitary, Feynman path sum and
               backward amplitudes for tiny circuits (pins for sv.py)
  philox.py    Philox4x32-10 counter-based generator (Salmon et al., SC'11)
  sampler.py   the modified frugal rejection sampler (Sec. II.A), step by step
  stats.py     linear XEB (Eq. 1), the sampler's output law and epsilon
               (Sec. II.A-C, Eqs. 3-5, 10), the fidelity bound (Eq. 9)
  partial.py   orthogonal slice decomposition psi = sum_i psi_i, norms R,
               SlicedVertexSelect and slice selection (Sec. I.A-C, Appendix B)
  spoof.py     linear-XEB spoofing: batch size, top selection, the XEB of the
               kept set and its expectation (Sec. III.B, Eqs. 11-12, Appendix A)

Only tests/, __graft_entry__.smoke() and bench.py's CPU-baseline leg may import
this package.  Nothing in the product path does.
"""
