"""Serving loop: a mix of requests overlapped on several streams gives, for
each request, bitwise the same amplitudes and samples as the request run alone;
admission never exceeds the HBM budget; over-budget and over-cost requests are
refused, not crashed; amplitudes match the oracle."""
import numpy as np
import pytest

from oracle import sv as osv

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import serve as s
    return s


def run_all(serve, reqs, **kw):
    srv = serve.Server(**kw)
    futs = [srv.submit(r) for r in reqs]
    res = [f.result(timeout=300) for f in futs]
    peak = srv.peak_in_use
    srv.shutdown()
    return res, peak


def mix(serve, n=10, seed=1):
    reqs = [r for _, r in serve.synthetic_requests(n, seed=seed, shapes=((3, 4), (4, 4), (4, 5)), cycles=(6, 10),
                                                   log2_amps=(6, 10), samples=(50, 200))]
    return reqs


def test_mix_equals_alone_and_matches_oracle(serve):
    """In the mix every request runs in work units of one slice group (a tiny
    unit time), alone in its default units: bitwise the same either way."""
    reqs = mix(serve)
    srv = serve.Server(n_streams=4, plan_workers=4, unit_seconds=1e-9)
    together = [f.result(timeout=300) for f in [srv.submit(r) for r in reqs]]
    units = srv.stats["units"]
    srv.shutdown()
    assert all(r.status == "ok" for r in together), [r.message for r in together]
    assert units > len(reqs)  # requests were split into several units
    for req, r in zip(reqs, together):
        alone, _ = run_all(serve, [req], n_streams=1, plan_workers=1)
        a = alone[0]
        assert serve.digest(a.amps) == serve.digest(r.amps), req.rid
        assert serve.digest(a.samples) == serve.digest(r.samples), req.rid
    # oracle parity on a few of them (complex64: rel-L2 <= 1e-5; bf16x3 requests are
    # checked at the split-mode bar 2e-4)
    for req, r in list(zip(reqs, together))[:4]:
        st = osv.simulate(req.text)
        for b, fb in enumerate(req.fixed_bits[:2]):
            ref = osv.batch_amplitudes(st, fb, req.open_qubits)
            err = np.linalg.norm(r.amps[b] - ref) / np.linalg.norm(ref)
            assert err <= (1e-5 if req.precision == 0 else 2e-4), (req.rid, err)


def test_admission_budget_and_refusals(serve):
    reqs = mix(serve, n=6, seed=2)
    # measure footprints, then serve under a budget that admits about two at once
    first, _ = run_all(serve, reqs, n_streams=4)
    fp = sorted(r.footprint for r in first)
    budget = fp[-1] + fp[-2]
    res, peak = run_all(serve, reqs, n_streams=4, hbm_budget=budget)
    assert all(r.status == "ok" for r in res)
    assert all(r.n_samples == req.n_samples for r, req in zip(res, reqs))  # 'ok' means the full count
    assert peak <= budget
    # a request larger than the whole budget is refused
    res, _ = run_all(serve, reqs[:2], n_streams=2, hbm_budget=fp[0] // 2)
    assert all(r.status == "refused" for r in res)
    # plan-cost cap
    res, _ = run_all(serve, reqs[:2], n_streams=2, plan_flops_cap=1.0)
    assert all(r.status == "refused" and "cap" in r.message for r in res)
