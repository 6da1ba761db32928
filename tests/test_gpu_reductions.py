"""FP64 probability sums on the GPU (the reductions of Sec. II.A and the sum in
the linear XEB of Eq. (1)), through the C-ABI, against their definitions.

  * Ragged shapes (one entry, a partial chunk, exactly one chunk, one entry
    past a chunk, several rows of several chunks, a long single row): each
    row's sum of (double)re^2 + (double)im^2 agrees with the oracle's
    definition to FP64 rounding order, and each row's XEB with the oracle's
    Eq. (1) on the same probabilities.
  * Repeated calls give the same bits; an empty row sums to 0, an XEB of an
    empty row and negative sizes are refused.
  * The squared norm of a 2^25-amplitude batch (the spoofing batch size).
  * The XEB of 2^19 amplitudes of bitstrings sampled from a random 16-qubit
    state: equal to the oracle's Eq. (1), and within 5 sigma of its
    expectation.
"""
import numpy as np
import pytest

from oracle import stats

pytestmark = pytest.mark.gpu

REL = 1e-13  # FP64, another summation order over at most 2^25 terms


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    return rqc, torch


def _amps(rng, n_rows, row_len, scale=1.0):
    a = (rng.standard_normal((n_rows, row_len, 2)) * scale).astype(np.float32)
    return a


def _ref_sums(a):
    p = a[..., 0].astype(np.float64) ** 2 + a[..., 1].astype(np.float64) ** 2
    return p, p.sum(axis=-1)


def _run(rqc, torch, a, n_qubits, with_xeb=True):
    n_rows, row_len = a.shape[0], a.shape[1]
    d = torch.from_numpy(a).cuda()
    sums = torch.full((n_rows,), -7.0, dtype=torch.float64, device="cuda")
    xeb = torch.full((n_rows,), -7.0, dtype=torch.float64, device="cuda") if with_xeb else None
    rqc.prob_sums(d, n_rows, row_len, n_qubits, sums, xeb)
    torch.cuda.synchronize()
    return sums.cpu().numpy(), (xeb.cpu().numpy() if with_xeb else None)


@pytest.mark.parametrize("n_rows,row_len", [(1, 1), (1, 63), (3, 8192), (2, 8193), (5, 20000), (1, 100003),
                                            (700, 64)])
def test_row_sums_and_xeb(lib, n_rows, row_len):
    rqc, torch = lib
    rng = np.random.default_rng(1000 * n_rows + row_len)
    n = 20
    a = _amps(rng, n_rows, row_len, scale=2.0 ** -10)
    print(f"prob_sums rows={n_rows} row_len={row_len}", flush=True)
    got, xeb = _run(rqc, torch, a, n)
    p, ref = _ref_sums(a)
    np.testing.assert_allclose(got, ref, rtol=REL, atol=0)
    for r in range(n_rows):
        x = stats.xeb(n, p[r])
        assert abs(xeb[r] - x) <= REL * (abs(x) + 1.0), (r, xeb[r], x)
    again, xeb2 = _run(rqc, torch, a, n)
    assert np.array_equal(again, got) and np.array_equal(xeb2, xeb)


def test_empty_and_refused(lib):
    rqc, torch = lib
    d = torch.zeros((3, 1, 2), dtype=torch.float32, device="cuda")
    sums = torch.full((3,), -7.0, dtype=torch.float64, device="cuda")
    rqc.prob_sums(d, 3, 0, 10, sums)
    torch.cuda.synchronize()
    assert sums.cpu().numpy().tolist() == [0.0, 0.0, 0.0]
    xeb = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(rqc.RqcError):
        rqc.prob_sums(d, 3, 0, 10, sums, xeb)
    with pytest.raises(rqc.RqcError):
        rqc.prob_sums(d, -1, 4, 10, sums)
    with pytest.raises(rqc.RqcError):
        rqc.prob_sums(d, 1, 1, 0, sums, xeb)
    rqc.prob_sums(d, 0, 5, 10, None)  # no rows: nothing to do


def test_full_batch_norm(lib):
    """The squared norm of one 2^25-amplitude batch (4096 chunks)."""
    rqc, torch = lib
    rng = np.random.default_rng(25)
    a = _amps(rng, 1, 1 << 25, scale=2.0 ** -13)
    print("prob_sums one row of 2^25", flush=True)
    got, _ = _run(rqc, torch, a, 30, with_xeb=False)
    _, ref = _ref_sums(a)
    assert abs(got[0] - ref[0]) <= REL * ref[0]


def test_xeb_of_porter_thomas_samples(lib):
    """Amplitudes of k bitstrings drawn from a random state's law p over 2^n
    outcomes: the XEB of Eq. (1) from the GPU sums equals the oracle's on the
    same probabilities, and lies within 5 sigma of its expectation
    2^n sum p^2 - 1 (sigma = sqrt(2/k): the variance of 2^n p under p is 2
    for a Porter-Thomas law)."""
    rqc, torch = lib
    n = 16
    rng = np.random.default_rng(16)
    psi = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    psi /= np.linalg.norm(psi)
    p = np.abs(psi) ** 2
    k = 1 << 19
    idx = rng.choice(1 << n, size=k, p=p / p.sum())
    a = np.stack([psi[idx].real, psi[idx].imag], axis=-1).astype(np.float32)[None]
    got, xeb = _run(rqc, torch, a, n)
    pf, _ = _ref_sums(a)
    x = stats.xeb(n, pf[0])
    assert abs(xeb[0] - x) <= REL * (abs(x) + 1.0)
    expect = (2.0 ** n) * float((p * p).sum()) - 1.0
    assert abs(xeb[0] - expect) <= 5 * np.sqrt(2.0 / k)
