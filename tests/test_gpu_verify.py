"""Verification of produced samples with exact amplitudes (Sec. III.A: the
samples' linear XEB needs the exact probability of every sampled bitstring).

Uncorrelated bitstrings each take a batch of their own with no open qubit;
the plan may keep its bitstring-independent subtrees in the global cache.

  * 512 seeded uniform bitstrings of a 20-qubit circuit: amplitudes within the
    complex64 bar of the oracle's state vector (relative L2 and element-wise),
    bitwise equal with and without the cache, and equal whatever the split of
    the bitstrings into calls.
  * Samples drawn by the library's sampler from correlated 2^12 batches of the
    same circuit, verified on the no-open-qubit plan: each verified amplitude
    agrees with the one the sampler saw (another contraction tree), and the
    samples' XEB from the verified probabilities (summed in FP64 on the GPU)
    equals the oracle's XEB of the same bitstrings and lies within 5 sigma of its expectation
    2^n sum p^2 - 1 (from the oracle's full vector).
"""
import math

import numpy as np
import pytest

import synthetic
from gpu_common import assert_close
from oracle import stats as ostats
from oracle import sv as osv

pytestmark = pytest.mark.gpu

TOL = 1e-5  # complex64 bar (relative L2)


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    return rqc, torch


@pytest.fixture(scope="module")
def circuit20():
    text = synthetic.circuit_text(4, 5, 12, 3)
    return text, osv.simulate(text)


def _verify(rqc, torch, plan, bits):
    out = torch.empty((len(bits), 1, 2), dtype=torch.float32, device="cuda")
    rqc.contract_amplitudes(plan, bits, out)
    torch.cuda.synchronize()
    return out


def test_uncorrelated_amplitudes(lib, circuit20):
    rqc, torch = lib
    text, sv = circuit20
    n = 20
    rng = np.random.default_rng(20)
    bits = [int(x) for x in rng.integers(0, 1 << n, 512)]
    c = rqc.load_circuit(text)
    cached = rqc.plan_create(c, [], n_sliced_target=4, max_log2_batched=2, path_seed=2, global_cache=1)
    plain = rqc.plan_create(c, [], path=rqc.plan_path(cached), sliced_legs=rqc.plan_sliced_legs(cached),
                            max_log2_batched=2)
    assert rqc.plan_info(cached)["n_open"] == 0
    print("verify 512 bitstrings, 20 qubits", flush=True)
    o1 = _verify(rqc, torch, plain, bits)
    o2 = _verify(rqc, torch, cached, bits)
    assert torch.equal(o1, o2)
    parts = [_verify(rqc, torch, cached, bits[a:b]) for a, b in ((0, 1), (1, 200), (200, 512))]
    assert torch.equal(torch.cat(parts), o2)
    a = o2.cpu().numpy()[:, 0, :]
    got = a[:, 0].astype(np.float64) + 1j * a[:, 1]
    ref = np.array([osv.batch_amplitudes(sv, b, [])[0] for b in bits])
    assert_close(got, ref, TOL, "uncorrelated amplitudes")


def test_sample_xeb_from_verified_amplitudes(lib, circuit20):
    rqc, torch = lib
    text, sv = circuit20
    n = 20
    open_q = list(range(8, 20))
    c = rqc.load_circuit(text)
    splan = rqc.plan_create(c, open_q, n_sliced_target=3, path_seed=1)
    out = torch.empty((1, 1 << 12, 2), dtype=torch.float32, device="cuda")
    samples = torch.zeros(64, dtype=torch.int64, device="cuda")
    drawn, seen = [], []
    call = 0
    while len(drawn) < 600:
        fb = [synthetic.fixed_bits(n, open_q, 7000 + call)]
        rqc.contract_amplitudes(splan, fb, out)
        n_out, _, _ = rqc.rejection_sample(out, fb, open_q, n, 64, samples, alpha=2.0, F_norm=1.0, seed=11,
                                           batch_index_base=call << 6)
        torch.cuda.synchronize()
        a = out.cpu().numpy()[0]
        for s in samples.cpu().numpy()[:n_out].astype(np.uint64):
            t = 0
            for j, q in enumerate(open_q):
                t |= int((int(s) >> q) & 1) << j
            drawn.append(int(s))
            seen.append(complex(a[t, 0], a[t, 1]))
        call += 1
    print(f"{len(drawn)} samples from {call} correlated batches", flush=True)
    vplan = rqc.plan_create(c, [], n_sliced_target=4, path_seed=5, global_cache=1)
    v = _verify(rqc, torch, vplan, drawn).cpu().numpy()[:, 0, :]
    amps = v[:, 0].astype(np.float64) + 1j * v[:, 1]
    assert_close(amps, np.array(seen), TOL, "verified vs sampled batch amplitudes")
    # the samples' XEB of Eq. (1) from the verified amplitudes, reduced on the GPU
    vd = torch.from_numpy(np.ascontiguousarray(v)).cuda()
    sum_d = torch.empty(1, dtype=torch.float64, device="cuda")
    xeb_d = torch.empty(1, dtype=torch.float64, device="cuda")
    rqc.prob_sums(vd, 1, len(drawn), n, sum_d, xeb_d)
    torch.cuda.synchronize()
    xeb_ver = float(xeb_d.item())
    p_ver = v[:, 0].astype(np.float64) ** 2 + v[:, 1].astype(np.float64) ** 2
    assert abs(xeb_ver - ostats.xeb(n, p_ver)) <= 1e-12 * (abs(xeb_ver) + 1.0)
    p_ora = np.array([abs(osv.batch_amplitudes(sv, b, [])[0]) ** 2 for b in drawn])
    xeb_ora = ostats.xeb(n, p_ora)
    assert abs(xeb_ver - xeb_ora) <= 1e-4 * max(1.0, abs(xeb_ora))
    p_all = np.abs(sv) ** 2
    expect = (2.0 ** n) * float((p_all ** 2).sum()) - 1.0
    sigma = float(np.std((2.0 ** n) * p_ora)) / math.sqrt(len(drawn))
    print(f"XEB of the samples {xeb_ver:.4f} (oracle {xeb_ora:.4f}), expected {expect:.4f} +- {sigma:.4f}",
          flush=True)
    assert abs(xeb_ver - expect) <= 5 * sigma + 0.02
