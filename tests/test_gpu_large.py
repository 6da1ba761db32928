"""The 53-qubit workload at its real shape (parity unpinned: no state vector of
53 qubits exists, so a property that holds at any size is checked instead).

Slices are a resolution of the identity (Sec. I), so the cross-slice sum is
additive over any split of the slice list into whole groups: the FP64 sum of
the first 16 slices in one call equals the sum of two calls over its halves,
up to FP64 reassociation.  The plan is the one the benchmark times: full
slicing to a 2^30-element bound on every intermediate, the largest launches
the library makes.
"""
import numpy as np
import pytest

import synthetic

pytestmark = pytest.mark.gpu


def test_large_slice_prefix_is_additive():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    n = cfg["rows"] * cfg["cols"] - len(cfg["removed"])
    open_q = list(cfg["open_qubits"])
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, max_log2_tensor=30, n_sliced_target=-1, max_log2_batched=30,
                        path_trials=4096)
    info = rqc.plan_info(p)
    assert info["n_qubits"] == 53 and info["max_log2_tensor"] <= 30
    group = 1 << info["n_batched"]
    ids = rqc.plan_slices(p, cap=16)
    assert len(ids) == 16 and 8 % group == 0
    fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED)]
    shape = (1, 1 << len(open_q), 2)
    amps = torch.empty(shape, dtype=torch.float32, device="cuda")
    full = torch.empty(shape, dtype=torch.float64, device="cuda")
    half = torch.empty_like(full)
    rqc.contract_amplitudes(p, fb, amps, full, slice_ids=ids)
    acc = torch.zeros_like(full)
    for part in (ids[:8], ids[8:]):
        rqc.contract_amplitudes(p, fb, amps, half, slice_ids=part)
        acc += half
    torch.cuda.synchronize()
    f = full.cpu().numpy()
    a = acc.cpu().numpy()
    assert np.isfinite(f).all()
    scale = np.abs(f).max()
    assert scale > 0
    assert np.abs(f - a).max() <= 1e-12 * scale
