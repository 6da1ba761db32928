"""GPU parity: the HIP path through the C-ABI against the FP64 oracle.

Bar (complex64 path): relative L2 error <= 1e-5 per returned batch; samples
bit-identical to the oracle's sampler for the same amplitudes and seed.
"""
import numpy as np
import pytest

import synthetic
from oracle import sampler as osamp
from oracle import sv as osv

from gpu_common import assert_close, circuit, oracle_batches

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def rqc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc as lib
    return lib


def run_amplitudes(rqc, text, open_qubits, fixed_list, **opts):
    import torch
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_qubits, **opts)
    out = torch.empty((len(fixed_list), 1 << len(open_qubits), 2), dtype=torch.float32, device="cuda")
    out64 = torch.empty((len(fixed_list), 1 << len(open_qubits), 2), dtype=torch.float64, device="cuda")
    rqc.contract_amplitudes(p, fixed_list, out, out64)
    torch.cuda.synchronize()
    a = out.cpu().numpy()
    a64 = out64.cpu().numpy()
    return a[..., 0] + 1j * a[..., 1], a64[..., 0] + 1j * a64[..., 1], rqc.plan_info(p), p


def test_tiny_all_open(rqc):
    cfg = synthetic.CONFIGS["tiny"]
    text = circuit(cfg["rows"], cfg["cols"], cfg["cycles"])
    amps, amps64, info, _ = run_amplitudes(rqc, text, cfg["open_qubits"], [0])
    ref = osv.simulate(text)
    assert_close(amps[0], ref, TOL)
    assert_close(amps64[0], ref, TOL)
    assert abs(np.sum(np.abs(amps[0]) ** 2) - 1) < 1e-5


@pytest.mark.parametrize("rows,cols,cycles,n_open,n_sliced,batched,seed", [
    (3, 3, 6, 4, 0, 28, 1),      # fixed bits, no slicing
    (4, 4, 8, 6, 3, 28, 2),      # slices carried as a batched mode
    (4, 4, 8, 6, 3, 1, 3),       # slices looped (at most one batched leg)
    (4, 5, 10, 8, 4, 2, 4),      # mixed looped / batched
    (5, 4, 12, 10, 5, 28, 5),    # larger intermediates (stream + GEMM steps)
])
def test_sliced_batches_match_oracle(rqc, rows, cols, cycles, n_open, n_sliced, batched, seed):
    text = circuit(rows, cols, cycles, seed=seed)
    n = rows * cols
    open_q = list(range(n - n_open, n))
    fixed = synthetic.fixed_bits_batch(n, open_q, 1000 + seed, 3)
    amps, amps64, info, _ = run_amplitudes(rqc, text, open_q, fixed, n_sliced_target=n_sliced,
                                           max_log2_batched=batched)
    assert info["n_sliced"] == n_sliced
    ref = oracle_batches(text, fixed, open_q)
    for b in range(len(fixed)):
        assert_close(amps[b], ref[b], TOL, f"batch {b}")


def test_vector_streaming_kernels_match_oracle(rqc):
    """The vector-ALU streaming kernels (LDS tile, long contracted index, generic),
    reached by switching the matrix-core forms off: parity on plans that use
    each of them, and the same tree with the matrix-core forms agrees."""
    seen = {}
    for rows, cols, cycles, seed, n_sliced in [(5, 5, 12, 3, 3), (4, 6, 14, 2, 3), (4, 5, 12, 1, 3)]:
        text = circuit(rows, cols, cycles, seed=seed)
        n = rows * cols
        open_q = list(range(n - 12, n))
        fixed = synthetic.fixed_bits_batch(n, open_q, 4000 + seed, 2)
        ref = oracle_batches(text, fixed, open_q)
        amps, _, info, p = run_amplitudes(rqc, text, open_q, fixed, n_sliced_target=n_sliced, path_seed=3,
                                          no_matrix_core_streams=1)
        sk = info["stream_kernels"]
        assert sk["mx"] == sk["mx2"] == sk["lk"] == 0, sk
        for k, v in sk.items():
            seen[k] = seen.get(k, 0) + v
        for b in range(2):
            assert_close(amps[b], ref[b], TOL, f"vector streams {rows}x{cols} batch {b}")
        amps_mx, _, info_mx, _ = run_amplitudes(rqc, text, open_q, fixed, path=rqc.plan_path(p),
                                                sliced_legs=rqc.plan_sliced_legs(p))
        assert info_mx["stream_kernels"]["mx"] > 0
        for b in range(2):
            assert_close(amps_mx[b], ref[b], TOL, f"matrix-core streams {rows}x{cols} batch {b}")
    assert seen["tile"] > 0 and seen["ky"] > 0 and seen["gen"] > 0, seen


def test_annealed_plan_matches_oracle(rqc):
    """A tree and slicing refined by simulated annealing (from a 16-trial
    search) contract to the oracle's amplitudes."""
    text = circuit(5, 5, 12, seed=8)
    open_q = list(range(13, 25))
    fixed = synthetic.fixed_bits_batch(25, open_q, 4100, 2)
    ref = oracle_batches(text, fixed, open_q)
    amps, _, info, p = run_amplitudes(rqc, text, open_q, fixed, n_sliced_target=3, path_trials=16, path_seed=2,
                                      anneal_iters=100_000)
    assert info["n_sliced"] == 3
    for b in range(2):
        assert_close(amps[b], ref[b], TOL, f"annealed plan batch {b}")


@pytest.mark.parametrize("cache", [0, 1])
def test_contract_in_group_units_is_bitwise_one_call(rqc, cache):
    """rqc_contract_groups over consecutive ranges of the default slice groups,
    then rqc_finalize_amplitudes, equals one rqc_contract_amplitudes call bit
    for bit (the FP64 running sum is carried in the accumulator), with and
    without the global cache; a range past the list is refused."""
    import torch
    text = circuit(4, 5, 12, seed=9)
    open_q = list(range(10, 20))
    fixed = synthetic.fixed_bits_batch(20, open_q, 4200, 3)
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, n_sliced_target=4, max_log2_batched=1, path_seed=4, global_cache=cache)
    info = rqc.plan_info(p)
    G = info["n_groups"]
    assert G >= 4
    shape = (3, 1 << len(open_q), 2)
    one = torch.empty(shape, dtype=torch.float32, device="cuda")
    one64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    rqc.contract_amplitudes(p, fixed, one, one64)
    acc = torch.full(shape, float("nan"), dtype=torch.float64, device="cuda")  # overwritten by the first unit
    cuts = [0, 1, G // 2, G - 1, G]
    for a, b in zip(cuts[:-1], cuts[1:]):
        rqc.contract_groups(p, a, b - a, fixed, acc)
    units = torch.empty(shape, dtype=torch.float32, device="cuda")
    units64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    rqc.finalize_amplitudes(p, acc, 3, units, units64)
    torch.cuda.synchronize()
    assert torch.equal(one, units) and torch.equal(one64, units64)
    ref = oracle_batches(text, fixed, open_q)
    a = units.cpu().numpy()
    for b in range(3):
        assert_close(a[b, :, 0] + 1j * a[b, :, 1], ref[b], TOL, f"group units batch {b}")
    with pytest.raises(rqc.RqcError):
        rqc.contract_groups(p, G - 1, 2, fixed, acc)


def test_single_amplitude_and_scalar_outputs(rqc):
    """No open qubit: each batch is one amplitude."""
    text = circuit(3, 3, 5, seed=6)
    fixed = [0, 5, 511, 300]
    amps, _, info, _ = run_amplitudes(rqc, text, [], fixed)
    state = osv.simulate(text)
    assert np.abs(amps[:, 0] - state[fixed]).max() <= TOL * np.abs(state).max() * 10


def test_gemm_steps_are_exercised(rqc):
    """A plan whose big steps run on the MFMA GEMM: parity and a non-zero GEMM share."""
    text = circuit(4, 5, 14, seed=7)
    open_q = list(range(8, 20))
    fixed = synthetic.fixed_bits_batch(20, open_q, 2000, 2)
    amps, _, info, _ = run_amplitudes(rqc, text, open_q, fixed, n_sliced_target=2, path_seed=3)
    ref = oracle_batches(text, fixed, open_q)
    for b in range(2):
        assert_close(amps[b], ref[b], TOL)
    assert info["gemm_flop_share"] > 0


def test_profiling_one_class_leaves_results_unchanged(rqc):
    """Timing only some kernel classes (rqc_plan_profile_classes): only their
    launches are recorded, with the same counts as when every class is timed,
    and the amplitudes are bitwise those of the unprofiled plan."""
    import torch
    text = circuit(4, 5, 14, seed=7)
    open_q = list(range(8, 20))
    fixed = synthetic.fixed_bits_batch(20, open_q, 2000, 2)
    c = rqc.load_circuit(text)
    base = rqc.plan_create(c, open_q, n_sliced_target=2, path_seed=3)
    opts = dict(path=rqc.plan_path(base), sliced_legs=rqc.plan_sliced_legs(base))
    outs, recs = [], []
    for prof, classes in ((0, None), (1, None), (1, ["gemm"]), (1, ["stream", "permute"])):
        p = rqc.plan_create(c, open_q, profile=prof, **opts)
        if classes:
            rqc.plan_profile_classes(p, classes)
        out = torch.empty((2, 1 << len(open_q), 2), dtype=torch.float32, device="cuda")
        rqc.contract_amplitudes(p, fixed, out)
        torch.cuda.synchronize()
        outs.append(out.cpu())
        recs.append(rqc.plan_profile_ops(p) if prof else [])
    for o in outs[1:]:
        assert torch.equal(o, outs[0])
    every = {}
    for r in recs[1]:
        every[r["cls"]] = every.get(r["cls"], 0) + r["launches"]
    assert every.get("gemm", 0) > 0 and len(every) > 2
    for got, classes in ((recs[2], {"gemm"}), (recs[3], {"stream", "permute"})):
        counts = {}
        for r in got:
            counts[r["cls"]] = counts.get(r["cls"], 0) + r["launches"]
        assert set(counts) <= classes and counts == {k: v for k, v in every.items() if k in classes}
    with pytest.raises(rqc.RqcError):
        rqc._check(rqc._lib.rqc_plan_profile_classes(base.handle, 1 << 8))  # no such class


def test_custom_slice_lists_sum_to_full(rqc):
    """Sum over any split of the slice list equals the full result (slices are a
    resolution of the identity, Sec. I)."""
    import torch
    text = circuit(4, 4, 8, seed=8)
    open_q = list(range(8, 16))
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, n_sliced_target=4, max_log2_batched=1)
    info = rqc.plan_info(p)
    nb = info["n_batched"]
    n_sl = info["n_slices"]
    ids = list(range(n_sl))
    legs = rqc.plan_sliced_legs(p)
    assert len(legs) == 4
    full = torch.empty((1, 256, 2), dtype=torch.float64, device="cuda")
    part = torch.empty_like(full)
    dummy = torch.empty((1, 256, 2), dtype=torch.float32, device="cuda")
    rqc.contract_amplitudes(p, [0], dummy, full)
    acc = torch.zeros_like(full)
    # batched legs are the low slice-id bits for a greedy plan: split into whole groups
    group = 1 << nb
    halves = [ids[: n_sl // 2], ids[n_sl // 2:]]
    for h in halves:
        assert len(h) % group == 0
        rqc.contract_amplitudes(p, [0], dummy, part, slice_ids=h)
        acc += part
    torch.cuda.synchronize()
    assert torch.allclose(acc, full, atol=1e-6)
    ref = oracle_batches(text, [0], open_q)[0]
    got = full.cpu().numpy()[0]
    assert_close(got[:, 0] + 1j * got[:, 1], ref, TOL)


def test_empty_slice_list_and_no_batches(rqc):
    """Degenerate calls: an empty slice list is the empty sum (all amplitudes
    exactly zero, both precisions); no batches writes nothing; a list that
    splits a batched group is refused before any launch."""
    import torch
    text = circuit(4, 4, 8, seed=8)
    open_q = list(range(8, 16))
    c = rqc.load_circuit(text)
    p = rqc.plan_create(c, open_q, n_sliced_target=4, max_log2_batched=1)
    nb = rqc.plan_info(p)["n_batched"]
    out = torch.full((2, 256, 2), float("nan"), dtype=torch.float32, device="cuda")
    out64 = torch.full((2, 256, 2), float("nan"), dtype=torch.float64, device="cuda")
    rqc.contract_amplitudes(p, [0, 3], out, out64, slice_ids=[])
    torch.cuda.synchronize()
    assert torch.equal(out, torch.zeros_like(out))
    assert torch.equal(out64, torch.zeros_like(out64))

    sentinel = torch.full((1, 256, 2), 7.0, dtype=torch.float32, device="cuda")
    rqc.contract_amplitudes(p, [], sentinel)
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())

    if nb > 0:
        with pytest.raises(rqc.RqcError, match="whole batched groups"):
            rqc.contract_amplitudes(p, [0], sentinel, slice_ids=[0])
    with pytest.raises(rqc.RqcError, match="beyond the sliced legs"):
        rqc.contract_amplitudes(p, [0], sentinel, slice_ids=[1 << 4])
    torch.cuda.synchronize()
    assert bool((sentinel == 7.0).all())


def test_sampler_batches_mode_bit_exact(rqc):
    import torch
    text = circuit(4, 4, 10, seed=9)
    open_q = list(range(4, 16))
    fixed = [0]
    amps, _, _, _ = run_amplitudes(rqc, text, open_q, fixed)
    A = amps.astype(np.complex64).reshape(-1, 64)
    dev = torch.from_numpy(np.stack([A.real, A.imag], -1).astype(np.float32)).cuda()
    out = torch.zeros(200, dtype=torch.int64, device="cuda")
    n_out, st, code = rqc.rejection_sample(dev, fixed, open_q, 16, 200, out, alpha=2.0, F_norm=1.0, seed=7,
                                           batch_index_base=5)
    ref, rst = osamp.sample_batches(A, 6, 1 << 10, 2.0, 1.0, 7, 5, 200)
    got = out.cpu().numpy()[:n_out].astype(np.uint64)
    exp = []
    for j, i in ref:
        t = (j << 6) | i
        bits = 0
        for b, q in enumerate(open_q):
            if (t >> b) & 1:
                bits |= 1 << q
        exp.append(bits)
    assert n_out == len(exp) and [int(x) for x in got] == exp
    assert st["accepted"] == rst["accepted"]
    assert abs(st["eps_J"] - rst["eps_j"]) <= 1e-12


@pytest.mark.parametrize("alpha", [2.0, 1.1])
def test_sampler_pick_mode_bit_exact(rqc, alpha):
    import torch
    cfg = synthetic.CONFIGS["tiny"]
    text = circuit(cfg["rows"], cfg["cols"], cfg["cycles"])
    amps, _, _, _ = run_amplitudes(rqc, text, cfg["open_qubits"], [0])
    a = amps[0].astype(np.complex64)
    f_norm = float(osamp.probabilities(a).sum())
    dev = torch.from_numpy(np.stack([a.real, a.imag], -1).astype(np.float32)).cuda()
    out = torch.zeros(1000, dtype=torch.int64, device="cuda")
    n_out, st, code = rqc.rejection_sample(dev, [0], cfg["open_qubits"], 12, 1000, out, alpha=alpha,
                                           F_norm=f_norm, seed=7, pick_steps=4000)
    ref, _ = osamp.sample_pick(a, 6, alpha, f_norm, 7, 1000, 4000)
    exp = [(j << 6) | i for j, i in ref]
    assert n_out == len(exp) == 1000
    assert [int(x) for x in out.cpu().numpy()] == exp


def test_sampler_short_status(rqc):
    import torch
    cfg = synthetic.CONFIGS["tiny"]
    text = circuit(cfg["rows"], cfg["cols"], cfg["cycles"])
    amps, _, _, _ = run_amplitudes(rqc, text, cfg["open_qubits"], [0])
    a = amps[0].astype(np.complex64)
    dev = torch.from_numpy(np.stack([a.real, a.imag], -1).astype(np.float32)).cuda()
    out = torch.zeros(1000, dtype=torch.int64, device="cuda")
    n_out, st, code = rqc.rejection_sample(dev, [0], cfg["open_qubits"], 12, 1000, out, pick_steps=100)
    assert code == rqc.ESHORT and n_out < 1000


@pytest.mark.parametrize("rows,cols,cycles,n_open,n_sliced,batched,seed", [
    (4, 4, 10, 6, 3, 1, 1),      # looped slices: one cache block per group
    (4, 5, 12, 8, 4, 2, 12),     # mixed looped / batched, GEMM steps
    (3, 4, 8, 12, 0, 28, 13),    # all qubits open: the whole contraction is cached
])
def test_global_cache_bitwise_equal(rqc, rows, cols, cycles, n_open, n_sliced, batched, seed):
    """The global cache (parts independent of the fixed bits computed once per
    slice group) changes no bit of any result, over successive calls with
    different fixed bits, and stays within the bar of the oracle."""
    import torch
    text = circuit(rows, cols, cycles, seed=seed)
    n = rows * cols
    open_q = list(range(n - n_open, n))
    c = rqc.load_circuit(text)
    opts = dict(n_sliced_target=n_sliced, max_log2_batched=batched, path_seed=seed)
    cached = rqc.plan_create(c, open_q, global_cache=1, **opts)
    # the uncached plan on the same tree and sliced legs (the planner's choice
    # differs with the cache, whose per-batch cost it minimises)
    plain = rqc.plan_create(c, open_q, path=rqc.plan_path(cached), sliced_legs=rqc.plan_sliced_legs(cached),
                            max_log2_batched=batched)
    info = rqc.plan_info(cached)
    assert info["cache_bytes"] > 0 and 0 < info["flops_cached"] <= info["flops_per_batch"]
    for call in range(3):
        fixed = synthetic.fixed_bits_batch(n, open_q, 3000 + 10 * seed + call, 2)
        o1 = torch.empty((2, 1 << n_open, 2), dtype=torch.float32, device="cuda")
        o2 = torch.empty_like(o1)
        rqc.contract_amplitudes(plain, fixed, o1)
        rqc.contract_amplitudes(cached, fixed, o2)
        torch.cuda.synchronize()
        assert torch.equal(o1, o2), call
        a = o2.cpu().numpy()
        ref = oracle_batches(text, fixed, open_q)
        for b in range(2):
            assert_close(a[b, :, 0] + 1j * a[b, :, 1], ref[b], TOL)
    # an explicit slice list bypasses the cache and still agrees bit for bit
    ids = list(range(info["n_slices"]))
    o1 = torch.empty((1, 1 << n_open, 2), dtype=torch.float32, device="cuda")
    o2 = torch.empty_like(o1)
    rqc.contract_amplitudes(plain, [5], o1, slice_ids=ids)
    rqc.contract_amplitudes(cached, [5], o2, slice_ids=ids)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


def test_global_cache_split_precision(rqc):
    """Cached and uncached plans agree bitwise in the bf16x3 mode too."""
    import torch
    text = circuit(4, 5, 12, seed=14)
    open_q = list(range(10, 20))
    c = rqc.load_circuit(text)
    cached = rqc.plan_create(c, open_q, global_cache=1, n_sliced_target=3, precision=rqc.BF16X3, path_seed=2)
    plain = rqc.plan_create(c, open_q, path=rqc.plan_path(cached), sliced_legs=rqc.plan_sliced_legs(cached),
                            precision=rqc.BF16X3)
    fixed = synthetic.fixed_bits_batch(20, open_q, 4000, 3)
    o1 = torch.empty((3, 1 << 10, 2), dtype=torch.float32, device="cuda")
    o2 = torch.empty_like(o1)
    rqc.contract_amplitudes(plain, fixed, o1)
    rqc.contract_amplitudes(cached, fixed, o2)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2)


@pytest.mark.parametrize("rows,cols,cycles,n_open,n_sliced,seed,precision,tol", [
    (4, 6, 14, 8, 4, 3, 0, TOL),      # a GEMM with K split in 2 ranges
    (5, 5, 14, 12, 5, 4, 0, TOL),     # K = 16384 split in 32 ranges
    (5, 5, 14, 12, 5, 4, 1, 2e-4),    # the same in bf16x3
])
def test_split_k_gemm_steps(rqc, rows, cols, cycles, n_open, n_sliced, seed, precision, tol):
    """Plans whose GEMMs have too few output tiles to fill the chip split K into
    ranges summed in order; parity with the oracle."""
    text = circuit(rows, cols, cycles, seed=seed)
    n = rows * cols
    open_q = list(range(n - n_open, n))
    fixed = synthetic.fixed_bits_batch(n, open_q, 5000 + seed, 2)
    amps, _, info, _ = run_amplitudes(rqc, text, open_q, fixed, n_sliced_target=n_sliced, path_seed=seed,
                                      precision=precision)
    ref = oracle_batches(text, fixed, open_q)
    for b in range(2):
        assert_close(amps[b], ref[b], tol, f"batch {b}")
