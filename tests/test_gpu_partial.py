"""Partial slicing on the GPU (Sec. I.A-I.C, Appendix B) against the oracle.

The library picks S by SlicedVertexSelect among its sliced legs, computes
R[i] = ||psi_i||^2 by contracting the doubled network C_1 C_1^* on the GPU,
keeps X by Alg. 1 and returns psi_X / sqrt(F).  The oracle recomputes S with
its own Alg. 2, R with projected state vectors, and psi_X as a sum of
projected state vectors.
"""
import math

import numpy as np
import pytest

import synthetic
from oracle import circuit as oc
from oracle import partial as opart
from oracle import sv as osv

from gpu_common import assert_close

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rqc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc as lib
    return lib


def partial_plan(rqc, text, open_q, n_sliced, f=None, count=None, batched=28):
    kw = dict(n_sliced_target=n_sliced, max_log2_batched=batched, path_seed=1)
    if f is not None:
        kw["target_fidelity"] = f
    if count is not None:
        kw["target_fidelity"] = 0.5
        kw["partial_count"] = count
    return rqc.plan_create(rqc.load_circuit(text), open_q, **kw)


@pytest.mark.parametrize("rows,cols,cycles,seed,n_sliced,f", [(4, 4, 10, 0, 10, 0.2), (4, 5, 12, 1, 12, 0.05)])
def test_partial_slicing_matches_oracle(rqc, rows, cols, cycles, seed, n_sliced, f):
    import torch
    text = synthetic.circuit_text(rows, cols, cycles, seed)
    n = rows * cols
    open_q = list(range(n - 8, n))
    p = partial_plan(rqc, text, open_q, n_sliced, f=f)
    info = rqc.plan_info(p)
    I = rqc.plan_sliced_legs(p)
    S, X, R = rqc.plan_partial(p)
    R = np.array(R)
    k = len(S)
    # Alg. 2 parity: the oracle's SlicedVertexSelect over the same sliced legs
    k0 = math.ceil(3 - math.log2(f))
    assert S == opart.sliced_vertex_select(oc.parse(text), I, k0)
    assert opart.is_antichain(oc.parse(text), S)
    # norms: GPU doubled network vs projected state vectors
    R_ref = opart.norms_R(text, S)
    assert abs(R.sum() - 1.0) <= 1e-5
    assert np.abs(R - R_ref).max() <= 1e-6
    # Alg. 1 invariants
    F = info["fidelity"]
    assert abs(F - R[X].sum()) <= 1e-12
    assert F >= f and F >= len(X) / 2 ** k - 1e-9
    assert len(X) <= math.ceil(f * 2 ** k)
    assert F - R[X[-1]] < f
    assert sorted(R, reverse=True)[: len(X)] == sorted(R[X].tolist(), reverse=True)
    assert info["n_slices"] == len(X) << (len(I) - k)
    # amplitudes: psi_X / sqrt(F) against the oracle's projected sum
    fixed = synthetic.fixed_bits_batch(n, open_q, 5000 + seed, 2)
    out = torch.empty((2, 256, 2), dtype=torch.float32, device="cuda")
    rqc.contract_amplitudes(p, fixed, out)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    got = got[..., 0] + 1j * got[..., 1]
    px = opart.psi_X(text, S, X)
    Fo = float(np.vdot(px, px).real)
    assert abs(Fo - R_ref[X].sum()) <= 1e-12
    for b in range(2):
        ref = osv.batch_amplitudes(px, fixed[b], open_q) / math.sqrt(Fo)
        assert_close(got[b], ref, 1e-5)


def test_partial_count_reading(rqc):
    """Keep exactly `count` top-R indices (the count reading of the 2^10-of-2^28 workload)."""
    text = synthetic.circuit_text(4, 4, 10, 2)
    p = partial_plan(rqc, text, list(range(8, 16)), 9, count=5)
    S, X, R = rqc.plan_partial(p)
    info = rqc.plan_info(p)
    assert len(X) == 5 and info["n_partial_kept"] == 5
    assert info["n_slices"] == 5 << (info["n_sliced"] - len(S))
    assert abs(info["fidelity"] - sum(R[i] for i in X)) <= 1e-12
