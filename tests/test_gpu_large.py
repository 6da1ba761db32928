"""The 53-qubit workload at its real shape: the plan the benchmark times
(partial slicing at f = 2^-18, 21 near-input partially sliced vertices,
intermediates bounded by 2^30 elements).

Pinned here:
  * the norm tensor R (2^21 entries, contracted on the GPU from the doubled
    network of Fig. 1) against the oracle's light-cone norms of the same S,
    entry by entry, and sum_i R[i] = 1 (Sec. I.A);
  * Alg. 1's X and F from that R (the oracle's selection), Eq. (2)'s
    F >= |X| / 2^k and |X| <= ceil(f 2^k);
  * slicing is a resolution of the identity (Sec. I): the FP64 sum over two
    batched groups of the share in one call equals the sum of two calls, and
    a group of slices equals, on the same tree, the sum over the same group
    with one more leg sliced (a different slicing, different launch shapes);
  * the streaming steps on 2^30-element tensors (the matrix-core kernel's
    64-bit addressed form) agree with the same slices on the vector kernels.
The amplitudes themselves are otherwise unpinned at 53 qubits (no state vector
of 53 qubits exists).
"""
import math
import types

import numpy as np
import pytest

import bench
import synthetic
from gpu_common import assert_close
from oracle import circuit as oc
from oracle import partial

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_15083_amd import rqc
    cfg = synthetic.CONFIGS["large"]
    text = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    open_q = list(cfg["open_qubits"])
    c = rqc.load_circuit(text)
    args = types.SimpleNamespace(path_trials=bench.LARGE_TRIALS, large_seeds=bench.LARGE_SEEDS,
                                 anneal_iters=bench.LARGE_ANNEAL)
    # the benchmark's plan: the stored result of its search when it matches
    stored = bench.stored_large_plan(text, args)
    path, legs, _ = stored if stored is not None else bench.plan_large(rqc, c, open_q, args)
    plan = rqc.plan_create(c, open_q, path=path, sliced_legs=legs, max_log2_tensor=30, max_log2_batched=30,
                           target_fidelity=bench.LARGE_F)
    return types.SimpleNamespace(rqc=rqc, torch=torch, text=text, open_q=open_q, c=c, path=path, legs=legs,
                                 plan=plan, n=53)


def test_norms_match_oracle_and_sum_to_one(setup):
    rqc = setup.rqc
    S, X, R = rqc.plan_partial(setup.plan)
    R = np.asarray(R)
    info = rqc.plan_info(setup.plan)
    k = len(S)
    assert k == 21 and R.size == 1 << 21 and info["max_log2_tensor"] <= 30
    c = oc.parse(setup.text)
    assert S == partial.sliced_vertex_select(c, setup.legs, 21) and partial.is_antichain(c, S)
    Ro = partial.norms_R_lightcone(setup.text, S)
    assert abs(R.sum() - 1.0) <= 1e-5
    assert np.abs(R - Ro).max() <= 1e-5 * Ro.max()
    # Alg. 1 on the GPU norms
    Xo, Fo = partial.select_slices(R, bench.LARGE_F)
    assert list(X) == Xo
    assert info["fidelity"] == pytest.approx(Fo, rel=1e-12)
    assert Fo >= len(X) / 2.0 ** k and len(X) <= math.ceil(bench.LARGE_F * 2 ** k)
    assert Fo >= bench.LARGE_F


def _share(setup):
    rqc = setup.rqc
    S, X, _ = rqc.plan_partial(setup.plan)
    info = rqc.plan_info(setup.plan)
    group = 1 << info["n_batched"]
    batched = []
    if info["n_batched"]:
        full = rqc.plan_slices(setup.plan, cap=group)
        bits = 0
        for sid in full:
            bits |= sid ^ full[0]
        batched = [v for t, v in enumerate(setup.legs) if (bits >> t) & 1]
    return bench.share_ids(setup.legs, S, X[0], 4 * group, batched), group


def test_share_is_additive(setup):
    rqc, torch = setup.rqc, setup.torch
    ids, group = _share(setup)
    fb = [synthetic.fixed_bits(setup.n, setup.open_q, synthetic.FIXED_BITS_SEED)]
    shape = (1, 1 << len(setup.open_q), 2)
    amps = torch.empty(shape, dtype=torch.float32, device="cuda")
    full = torch.empty(shape, dtype=torch.float64, device="cuda")
    half = torch.empty_like(full)
    two = ids[:2 * group]
    rqc.contract_amplitudes(setup.plan, fb, amps, full, slice_ids=two)
    acc = torch.zeros_like(full)
    for part in (two[:group], two[group:]):
        rqc.contract_amplitudes(setup.plan, fb, amps, half, slice_ids=part)
        acc += half
    torch.cuda.synchronize()
    f, a = full.cpu().numpy(), acc.cpu().numpy()
    assert np.isfinite(f).all() and np.abs(f).max() > 0
    assert np.abs(f - a).max() <= 1e-12 * np.abs(f).max()


def test_another_slicing_of_the_same_tree_agrees(setup):
    rqc, torch = setup.rqc, setup.torch
    ids, group = _share(setup)
    # one more leg sliced on the same tree: an internal variable of the
    # circuit's middle that is not sliced yet
    extra = next(v for v in range(560, 1100) if v not in setup.legs)
    legs_b = list(setup.legs) + [extra]
    # every leg looped (no batched mode), so any list of slice ids is whole groups
    plan_b = rqc.plan_create(setup.c, setup.open_q, path=setup.path, sliced_legs=legs_b, max_log2_batched=1)
    S, _, _ = rqc.plan_partial(setup.plan)
    info = rqc.plan_info(setup.plan)
    F = info["fidelity"]
    fb = [synthetic.fixed_bits(setup.n, setup.open_q, synthetic.FIXED_BITS_SEED + 1)]
    shape = (1, 1 << len(setup.open_q), 2)
    amps = torch.empty(shape, dtype=torch.float32, device="cuda")
    a64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    b64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    sel = ids[:group]
    rqc.contract_amplitudes(setup.plan, fb, amps, a64, slice_ids=sel)
    top = 1 << len(setup.legs)
    info_b = rqc.plan_info(plan_b)
    assert info_b["n_batched"] == 0 and info_b["n_sliced"] == len(legs_b)
    ids_b = sorted(set(sel) | {s | top for s in sel})
    rqc.contract_amplitudes(plan_b, fb, amps, b64, slice_ids=ids_b)
    torch.cuda.synchronize()
    a = a64.cpu().numpy()
    b = b64.cpu().numpy() / math.sqrt(F)  # plan_b is full slicing (F = 1); the plan divides by sqrt(F)
    scale = np.abs(a).max()
    assert scale > 0
    assert np.abs(a - b).max() <= 2e-5 * scale


def test_matrix_core_and_vector_streams_agree_at_full_size(setup):
    """Streaming steps on 2^30-element tensors in the 64-bit addressed
    matrix-core form ("mx-wide"), on the searched 53-qubit plan before
    annealing (which has such steps): the same tree and slices with every
    streaming step on the vector kernels (checked against the oracle at small
    sizes) agree to FP32 rounding."""
    rqc, torch = setup.rqc, setup.torch
    args = types.SimpleNamespace(path_trials=bench.LARGE_TRIALS, large_seeds=bench.LARGE_SEEDS, anneal_iters=0)
    path, legs, _ = bench.plan_large(rqc, setup.c, setup.open_q, args)
    plan = rqc.plan_create(setup.c, setup.open_q, path=path, sliced_legs=legs, max_log2_tensor=30,
                           max_log2_batched=30, target_fidelity=bench.LARGE_F)
    desc = rqc.plan_describe(plan)
    assert " mx-wide " in desc, "the searched plan has no wide matrix-core streaming step"
    plan_v = rqc.plan_create(setup.c, setup.open_q, path=path, sliced_legs=legs, max_log2_tensor=30,
                             max_log2_batched=30, target_fidelity=bench.LARGE_F, no_matrix_core_streams=1)
    assert " mx-wide " not in rqc.plan_describe(plan_v) and " mx " not in rqc.plan_describe(plan_v)
    assert rqc.plan_info(plan_v)["fidelity"] == rqc.plan_info(plan)["fidelity"]
    S, X, _ = rqc.plan_partial(plan)
    info = rqc.plan_info(plan)
    group = 1 << info["n_batched"]
    batched = []
    if info["n_batched"]:
        full = rqc.plan_slices(plan, cap=group)
        bits = 0
        for sid in full:
            bits |= sid ^ full[0]
        batched = [v for t, v in enumerate(legs) if (bits >> t) & 1]
    sel = bench.share_ids(legs, S, X[0], 2 * group, batched)
    fb = [synthetic.fixed_bits(setup.n, setup.open_q, synthetic.FIXED_BITS_SEED + 2)]
    shape = (1, 1 << len(setup.open_q), 2)
    amps = torch.empty(shape, dtype=torch.float32, device="cuda")
    a64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    v64 = torch.empty(shape, dtype=torch.float64, device="cuda")
    rqc.contract_amplitudes(plan, fb, amps, a64, slice_ids=sel)
    rqc.contract_amplitudes(plan_v, fb, amps, v64, slice_ids=sel)
    torch.cuda.synchronize()
    a = a64.cpu().numpy()[0]
    v = v64.cpu().numpy()[0]
    a = a[:, 0] + 1j * a[:, 1]
    v = v[:, 0] + 1j * v[:, 1]
    assert np.abs(a).max() > 0
    assert_close(a, v, 1e-5, "matrix-core vs vector streams")
