"""The allocation-free sampling entry point (rqc_rejection_sample_static) against
rqc_rejection_sample, through the C-ABI: two calls in a row on the fixed device
array, the second with a smaller input, each bit-identical to the allocating
entry point on the same amplitudes (samples, count and statistics); pick mode
likewise; a call that needs more than the array holds is refused on the host."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

N_QUBITS = 20
OPEN = list(range(12))


def _amps(torch, n_batches, seed):
    # Porter-Thomas-like amplitudes, normalised over the whole 2^20 space
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((n_batches, 1 << len(OPEN), 2)).astype(np.float32)
    a *= np.float32(1.0 / np.sqrt(2.0 * (1 << N_QUBITS)))
    return torch.from_numpy(a).cuda()


def _fixed(n_batches, seed):
    rng = np.random.default_rng(seed)
    mask = ((1 << N_QUBITS) - 1) & ~((1 << len(OPEN)) - 1)
    return [int(x) & mask for x in rng.integers(0, 1 << N_QUBITS, size=n_batches)]


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    return rqc, torch


def _both(rqc, torch, amps, fixed, n_samples, base, **kw):
    outs = []
    for fn in (rqc.rejection_sample, rqc.rejection_sample_static):
        samples = torch.full((max(n_samples, 1),), -1, dtype=torch.int64, device="cuda")
        n_out, st, code = fn(amps, fixed, OPEN, N_QUBITS, n_samples, samples, alpha=2.0, F_norm=1.0, seed=7,
                             batch_index_base=base, **kw)
        torch.cuda.synchronize()
        outs.append((n_out, st, code, samples.cpu().numpy()[:n_out].copy()))
    return outs


def test_static_scratch_matches_allocating_entry_point(lib):
    rqc, torch = lib
    # first call: 8 batches (512 sub-batches); second: 2 batches, fewer samples
    for n_batches, n_samples, seed in ((8, 200, 11), (2, 40, 12)):
        amps = _amps(torch, n_batches, seed)
        fixed = _fixed(n_batches, seed)
        (n1, st1, c1, s1), (n2, st2, c2, s2) = _both(rqc, torch, amps, fixed, n_samples, base=seed << 20)
        print(f"batches {n_batches}: {n1} samples, status {c1}", flush=True)
        assert n1 > 0 and (n1, c1) == (n2, c2)
        assert st1 == st2
        assert np.array_equal(s1, s2)


def test_static_scratch_pick_mode(lib):
    rqc, torch = lib
    n = 12
    rng = np.random.default_rng(5)
    a = rng.standard_normal((1, 1 << n, 2)).astype(np.float32) * np.float32(1.0 / np.sqrt(2.0 * (1 << n)))
    amps = torch.from_numpy(a).cuda()
    f_norm = float((a.astype(np.float64) ** 2).sum())
    outs = []
    for fn in (rqc.rejection_sample, rqc.rejection_sample_static):
        samples = torch.full((300,), -1, dtype=torch.int64, device="cuda")
        n_out, st, code = fn(amps, [0], list(range(n)), n, 300, samples, alpha=2.0, F_norm=f_norm, seed=3,
                             pick_steps=2000)
        torch.cuda.synchronize()
        outs.append((n_out, st, code, samples.cpu().numpy()[:n_out].copy()))
    assert outs[0][0] == 300 and outs[0][:3] == outs[1][:3]
    assert np.array_equal(outs[0][3], outs[1][3])


def test_static_scratch_refuses_oversized_calls(lib):
    rqc, torch = lib
    # 8193 batches of 64 sub-batches need 16 * 524352 bytes of results alone
    n_batches = (rqc.SAMPLE_STATIC_SCRATCH_BYTES // 16) // 64 + 1
    amps = torch.zeros((n_batches, 1 << len(OPEN), 2), dtype=torch.float32, device="cuda")
    samples = torch.zeros(16, dtype=torch.int64, device="cuda")
    with pytest.raises(rqc.RqcError) as e:
        rqc.rejection_sample_static(amps, [0] * n_batches, OPEN, N_QUBITS, 16, samples)
    assert e.value.status == rqc.EINVAL and "fixed array" in str(e.value)
    # the array still serves a call after the refusal
    amps = _amps(torch, 1, 3)
    (n1, st1, _, s1), (n2, st2, _, s2) = _both(rqc, torch, amps, _fixed(1, 3), 10, base=0)
    assert n1 == n2 and st1 == st2 and np.array_equal(s1, s2)
