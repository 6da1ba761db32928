"""The 30-qubit workloads at full size, planned as the benchmark plans them
(65536 randomised greedy trials, seed 0, the fastest of four estimated trees
timed on the GPU), against the oracle's stored FP64 amplitudes (tests/golden,
written from the oracle's full state vector only).

Bar: relative L2 error <= 1e-5 (the complex64 bar) for the complex64 output
and for the FP64 copy of the same sum, on both stored batches (two fixed-bit
seeds) of each workload.  The batch sampler (Sec. II.A), called on those
complex64 amplitudes as the benchmark calls it, returns bitstrings identical
to the oracle sampler's on the same amplitudes.
"""
import os

import numpy as np
import pytest

import synthetic
from gpu_common import rel_l2
from oracle import sampler as osamp

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-5


@pytest.mark.parametrize("name", ["mid", "precision"])
def test_full_size_batches_match_stored_oracle(name):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    cfg = synthetic.CONFIGS[name]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    open_q = list(cfg["open_qubits"])
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, n_sliced_target=cfg["n_sliced"], path_trials=65536, path_seed=0,
                        autotune=4)
    info = rqc.plan_info(p)
    n = info["n_qubits"]
    assert info["n_sliced"] == cfg["n_sliced"]
    shape = (1, 1 << len(open_q), 2)
    out = torch.empty(shape, dtype=torch.float32, device="cuda")
    out64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    for call in range(2):
        ref = np.load(os.path.join(HERE, "golden", f"{name}_seed0_call{call}.npy"))
        fb = [synthetic.fixed_bits(n, open_q, synthetic.FIXED_BITS_SEED + call)]
        rqc.contract_amplitudes(p, fb, out, out64)
        torch.cuda.synchronize()
        a = out.cpu().numpy()[0]
        a64 = out64.cpu().numpy()[0]
        got = a[:, 0].astype(np.float64) + 1j * a[:, 1]
        got64 = a64[:, 0] + 1j * a64[:, 1]
        assert rel_l2(got, ref) <= TOL, (name, call, rel_l2(got, ref))
        assert rel_l2(got64, ref) <= TOL, (name, call, rel_l2(got64, ref))

        o = len(open_q)
        n_sub = 1 << (o - 6)
        base = call << (o - 6)
        samples = torch.zeros(n_sub, dtype=torch.int64, device="cuda")
        n_out, st, _ = rqc.rejection_sample(out, fb, open_q, n, n_sub, samples, alpha=cfg["alpha"], F_norm=1.0,
                                            seed=synthetic.SAMPLER_SEED, batch_index_base=base)
        A = (a[:, 0] + 1j * a[:, 1]).astype(np.complex64).reshape(-1, 64)
        picks, rst = osamp.sample_batches(A, 6, 1 << (n - 6), cfg["alpha"], 1.0, synthetic.SAMPLER_SEED, base,
                                          n_sub)
        open_mask = sum(1 << q for q in open_q)
        exp = []
        for j, i in picks:
            t = (j << 6) | i
            bits = fb[0] & ~open_mask
            for b, q in enumerate(open_q):
                if (t >> b) & 1:
                    bits |= 1 << q
            exp.append(bits)
        got_s = [int(x) for x in samples.cpu().numpy()[:n_out].astype(np.uint64)]
        assert n_out == len(exp) and got_s == exp, (name, call)
        assert n_out > 0 and st["accepted"] == rst["accepted"]
