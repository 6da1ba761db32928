"""CPU tests of the serving loop's host pieces (request mix, digests)."""
import numpy as np

from paper_2112_15083_amd import serve


def test_request_mix_is_seeded_and_well_formed():
    a = serve.synthetic_requests(20, seed=3, rate=5.0)
    b = serve.synthetic_requests(20, seed=3, rate=5.0)
    assert [(t, r.text, r.fixed_bits, r.n_samples, r.precision) for t, r in a] == \
           [(t, r.text, r.fixed_bits, r.n_samples, r.precision) for t, r in b]
    times = [t for t, _ in a]
    assert times == sorted(times) and times[0] > 0
    for _, r in a:
        assert len(r.open_qubits) >= 6 and max(r.open_qubits) < r.n_qubits
        open_mask = sum(1 << q for q in r.open_qubits)
        assert all(fb & open_mask == 0 for fb in r.fixed_bits)
        if r.n_samples:
            # enough sub-batches for alpha = 2 on average
            assert len(r.fixed_bits) << (len(r.open_qubits) - 6) >= 2 * r.n_samples
        assert r.precision in (0, 1)


def test_digest_distinguishes_bits():
    x = np.arange(8, dtype=np.complex128)
    y = x.copy()
    y[3] = np.nextafter(y[3].real, 10) + 0j
    assert serve.digest(x) == serve.digest(x.copy()) != serve.digest(y)
    assert serve.digest(None) == ""
