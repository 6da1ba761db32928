"""End-to-end precision modes: the same plan in complex64, bf16x3 and fp16x3,
with the error against the FP64 oracle stated per mode (the split modes only
change GEMM steps with K >= 16)."""
import numpy as np
import pytest

import synthetic
from oracle import sampler as osamp

from gpu_common import assert_close, circuit, oracle_batches, rel_l2

pytestmark = pytest.mark.gpu

BARS = {"C64": 1e-5, "BF16X3": 2e-4, "FP16X3": 1e-5}


@pytest.fixture(scope="module")
def rqc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc as lib
    return lib


@pytest.mark.parametrize("rows,cols,cycles,seed,n_sliced", [(5, 5, 12, 3, 3), (4, 6, 14, 2, 3)])
def test_precision_modes_against_oracle(rqc, rows, cols, cycles, seed, n_sliced):
    import torch
    text = circuit(rows, cols, cycles, seed=seed)
    n = rows * cols
    open_q = list(range(n - 12, n))
    fixed = synthetic.fixed_bits_batch(n, open_q, 3000 + seed, 2)
    ref = oracle_batches(text, fixed, open_q)
    c = rqc.load_circuit(text)
    errs = {}
    amps = {}
    for mode in ("C64", "BF16X3", "FP16X3"):
        p = rqc.plan_create(c, open_q, n_sliced_target=n_sliced, path_seed=3, precision=getattr(rqc, mode))
        info = rqc.plan_info(p)
        assert info["gemm_flop_share"] > 0.3
        out = torch.empty((2, 4096, 2), dtype=torch.float32, device="cuda")
        rqc.contract_amplitudes(p, fixed, out)
        torch.cuda.synchronize()
        a = out.cpu().numpy()
        a = a[..., 0] + 1j * a[..., 1]
        amps[mode] = a
        errs[mode] = max(rel_l2(a[b], ref[b]) for b in range(2))
        for b in range(2):
            assert_close(a[b], ref[b], BARS[mode], f"{mode} batch {b}")
        assert errs[mode] <= BARS[mode], (mode, errs)
    # the split modes really take another arithmetic route
    assert not np.array_equal(amps["C64"], amps["BF16X3"])
    print("rel-L2 vs FP64:", {k: f"{v:.2e}" for k, v in errs.items()})
