"""CPU tests of the C-ABI library: it loads, exports every declared symbol, and
its host-side planner (dry-run mode, no GPU) behaves as documented."""
import os
import re

import pytest

import synthetic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def rqc():
    from paper_2112_15083_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    from paper_2112_15083_amd import rqc as lib
    return lib


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "rqc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rqc_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(rqc):
    import ctypes
    lib = ctypes.CDLL(rqc.LIB_PATH)
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert set(syms) == set(rqc.EXPORTS)


def test_one_hip_runtime_whatever_the_import_order(rqc):
    """The binding loads torch's HIP runtime before the library, so importing the
    binding first and torch afterwards still maps a single libamdhip64 (two
    runtimes in one process do not share devices, streams or pointers)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_2112_15083_amd import rqc\nimport torch\n"
            "print(len({l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.strip().splitlines()[-1] == "1"


def test_parse_errors_are_reported(rqc):
    with pytest.raises(rqc.RqcError) as e:
        rqc.load_circuit("qubits 2\nsx 0 5\n")
    assert e.value.status == rqc.EPARSE
    with pytest.raises(rqc.RqcError) as e:
        rqc.load_circuit("qubits 2\nfoo 0 1\n")
    assert "line 2" in str(e.value)
    with pytest.raises(rqc.RqcError):
        rqc.load_circuit("sx 0 0\n")


def test_circuit_info_counts_variables(rqc):
    t = synthetic.circuit_text(3, 4, 8, 0)
    info = rqc.circuit_info(rqc.load_circuit(t))
    # 12 inputs + one variable per single-qubit gate (fSim(pi/2) adds none)
    assert info == dict(n_qubits=12, n_variables=12 + 12 * 8, n_gates=t.count("\nsx") + t.count("\nsy")
                        + t.count("\nsw") + t.count("\nfsim"))


def test_dry_run_plans(rqc):
    for name, ns in (("tiny", 0), ("mid", 6)):
        cfg = synthetic.CONFIGS[name]
        t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
        p = rqc.plan_create(rqc.load_circuit(t), cfg["open_qubits"], dry_run=1, n_sliced_target=ns)
        info = rqc.plan_info(p)
        assert info["n_sliced"] == ns and info["n_slices"] == 1 << ns
        assert info["n_open"] == len(cfg["open_qubits"])
        assert info["flops_per_batch"] > 0
        legs = rqc.plan_sliced_legs(p)
        assert len(legs) == ns and len(set(legs)) == ns
        # sliced legs are internal variables: not inputs, not outputs
        assert all(v >= cfg["rows"] * cfg["cols"] for v in legs)


def test_global_cache_plan_report(rqc):
    """The global cache covers exactly the work that does not depend on the
    fixed bits: everything when all qubits are open, part of it otherwise, and
    it holds one block per slice group plus a spare."""
    cfg = synthetic.CONFIGS["tiny"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"])
    info = rqc.plan_info(rqc.plan_create(rqc.load_circuit(t), cfg["open_qubits"], dry_run=1, global_cache=1))
    assert info["flops_cached"] == info["flops_per_batch"]
    assert info["cache_bytes"] == 2 * 8 * 2 ** 12  # the final 2^12 tensor, one group + spare
    t = synthetic.circuit_text(4, 4, 10, 1)
    c = rqc.load_circuit(t)
    cached = rqc.plan_create(c, list(range(10, 16)), dry_run=1, n_sliced_target=3, max_log2_batched=1,
                             path_seed=1, global_cache=1)
    info = rqc.plan_info(cached)
    # the same tree without the cache (the planner's own choice differs with it)
    plain = rqc.plan_info(rqc.plan_create(c, list(range(10, 16)), dry_run=1, path=rqc.plan_path(cached),
                                          sliced_legs=rqc.plan_sliced_legs(cached), max_log2_batched=1))
    assert plain["cache_bytes"] == 0 and plain["flops_cached"] == 0
    assert 0 < info["flops_cached"] < info["flops_per_batch"] == plain["flops_per_batch"]
    assert info["cache_bytes"] % (8 * (info["n_groups"] + 1)) == 0


def test_plan_path_round_trip(rqc):
    """A plan's path and sliced legs rebuild the same plan."""
    t = synthetic.circuit_text(4, 5, 12, 12)
    c = rqc.load_circuit(t)
    p1 = rqc.plan_create(c, list(range(12, 20)), dry_run=1, n_sliced_target=4, path_seed=12)
    path = rqc.plan_path(p1)
    n_leaves = len(path) + 1
    used = set()
    for s_, (a, b) in enumerate(path):  # SSA pairs: each tensor used once, results numbered in order
        assert a != b and a < n_leaves + s_ and b < n_leaves + s_ and a not in used and b not in used
        used.update((a, b))
    p2 = rqc.plan_create(c, list(range(12, 20)), dry_run=1, path=path, sliced_legs=rqc.plan_sliced_legs(p1))
    i1, i2 = rqc.plan_info(p1), rqc.plan_info(p2)
    assert rqc.plan_path(p2) == path
    for k in ("flops_per_batch", "n_batched", "n_slices", "max_log2_tensor", "n_launches"):
        assert i1[k] == i2[k], k


def test_stream_fusion_report(rqc):
    """On the 30-qubit workload's tree (tests/data/mid_tree.json) the planner
    fuses the two pairs of consecutive rank-28 streaming steps, cutting their
    HBM bytes; the opt-out keeps every step separate with the same flops."""
    import json
    import os
    tree = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "mid_tree.json")))
    cfg = synthetic.CONFIGS["mid"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    c = rqc.load_circuit(t)
    f = rqc.plan_info(rqc.plan_create(c, cfg["open_qubits"], dry_run=1, path=tree["path"], sliced_legs=tree["sliced"]))
    u = rqc.plan_info(rqc.plan_create(c, cfg["open_qubits"], dry_run=1, path=tree["path"], sliced_legs=tree["sliced"],
                                      no_stream_fusion=1))
    assert f["n_fused"] == 2 and u["n_fused"] == 0
    assert f["flops_per_batch"] == u["flops_per_batch"]
    assert f["n_launches"] == u["n_launches"] - 2
    # each fused pair drops one rank-28 intermediate written and read back (2 x 2 GiB)
    assert u["bytes_per_batch"] - f["bytes_per_batch"] >= 2 * 2 * 8 * 2 ** 28 * 0.99 * f["n_groups"]
    assert f["est_seconds"] < u["est_seconds"]


def test_memory_target_slicing(rqc):
    cfg = synthetic.CONFIGS["mid"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"])
    p = rqc.plan_create(rqc.load_circuit(t), cfg["open_qubits"], dry_run=1, max_log2_tensor=20,
                        n_sliced_target=-1, max_log2_batched=20)
    info = rqc.plan_info(p)
    assert info["max_log2_tensor"] <= 20
    assert info["n_sliced"] > 0


def test_invalid_plan_arguments(rqc):
    t = synthetic.circuit_text(3, 3, 4, 0)
    c = rqc.load_circuit(t)
    with pytest.raises(rqc.RqcError):
        rqc.plan_create(c, [0, 0], dry_run=1)
    with pytest.raises(rqc.RqcError):
        rqc.plan_create(c, [9], dry_run=1)
    with pytest.raises(rqc.RqcError):  # an input variable cannot be sliced
        rqc.plan_create(c, [0], dry_run=1, sliced_legs=[0])
    with pytest.raises(rqc.RqcError):  # a path that does not contract everything
        rqc.plan_create(c, [0], dry_run=1, path=[(0, 1)])


def test_user_path_and_legs_are_used(rqc):
    t = synthetic.circuit_text(2, 2, 3, 0)
    c = rqc.load_circuit(t)
    n_g = rqc.circuit_info(c)["n_gates"]
    # left-deep order over the gate tensors
    path = [(0, 1)] + [(n_g + s, s + 2) for s in range(n_g - 2)]
    p = rqc.plan_create(c, [0, 1], dry_run=1, path=path, sliced_legs=[5])
    info = rqc.plan_info(p)
    assert info["n_steps"] == n_g - 1 and rqc.plan_sliced_legs(p) == [5]


def test_annealing_refines_a_weak_search(rqc):
    """Simulated annealing of tree and slicing (the optimiser Sec. I names for
    T and I) from 64-trial searches of the 30-qubit circuit: the searched trees
    stay candidates, so the kept plan is never estimated slower; from at least
    one of three search seeds it is estimated 10 % faster with fewer flops; it
    keeps the 6 prescribed sliced legs and round-trips through its path."""
    cfg = synthetic.CONFIGS["mid"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    c = rqc.load_circuit(t)
    gains = []
    for seed in (1, 2, 3):
        base = rqc.plan_create(c, cfg["open_qubits"], n_sliced_target=6, path_trials=64, path_seed=seed, dry_run=1)
        ann = rqc.plan_create(c, cfg["open_qubits"], n_sliced_target=6, path_trials=64, path_seed=seed, dry_run=1,
                              anneal_iters=200_000)
        bi, ai = rqc.plan_info(base), rqc.plan_info(ann)
        assert ai["n_sliced"] == 6
        assert ai["est_seconds"] <= bi["est_seconds"]
        if ai["est_seconds"] < 0.9 * bi["est_seconds"]:
            assert ai["flops_per_batch"] < bi["flops_per_batch"]
            gains.append(seed)
        again = rqc.plan_create(c, cfg["open_qubits"], path=rqc.plan_path(ann),
                                sliced_legs=rqc.plan_sliced_legs(ann), dry_run=1)
        assert rqc.plan_info(again)["flops_per_batch"] == ai["flops_per_batch"]
    assert gains


def test_plan_describe_lists_every_launch(rqc):
    """rqc_plan_describe: one line per op of the launch program, with the
    kernel each streaming step runs on and the GEMM shapes."""
    cfg = synthetic.CONFIGS["mid"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    p = rqc.plan_create(rqc.load_circuit(t), cfg["open_qubits"], n_sliced_target=6, path_seed=1, dry_run=1)
    info = rqc.plan_info(p)
    lines = rqc.plan_describe(p).splitlines()
    ops = [ln.split() for ln in lines[1:]]
    assert lines[0].startswith("#") and len(ops) == info["n_launches"] - 2  # + leaf select and accumulate
    assert [int(o[0]) for o in ops] == list(range(len(ops)))
    kinds = {o[1] for o in ops}
    assert kinds <= {"small", "stream", "permute", "gemm"} and "gemm" in kinds and "stream" in kinds
    streams = [o[2] for o in ops if o[1] == "stream"]
    sk = info["stream_kernels"]
    for k in ("mx2", "lk", "tile"):
        assert streams.count(k) == sk[k]
    assert streams.count("mx") + streams.count("mx-wide") == sk["mx"]
    flops = sum(float(o[4]) for o in ops)
    assert abs(flops * info["n_groups"] - info["flops_per_batch"]) <= 1e-6 * info["flops_per_batch"]

def test_gemm_feeding_a_fused_pair_inserts_its_leg(rqc):
    """On the 30-qubit plan the GEMM whose result is the first fused pair's
    large operand writes that result with one leg the pair contracts placed
    at position 3 among its N legs (c_ins=3/1), so the pair's tile covers the
    operand's four lowest bits (a whole 128-byte line); no other GEMM does."""
    cfg = synthetic.CONFIGS["mid"]
    t = synthetic.circuit_text(cfg["rows"], cfg["cols"], cfg["cycles"], cfg["seed"], cfg["removed"])
    p = rqc.plan_create(rqc.load_circuit(t), cfg["open_qubits"], n_sliced_target=6, path_trials=65536, dry_run=1)
    lines = rqc.plan_describe(p).splitlines()[1:]
    ins = [ln.split() for ln in lines if "c_ins=" in ln]
    assert len(ins) == 1 and ins[0][1] == "gemm" and ins[0][-1] == "c_ins=3/1"
    nxt = [ln.split() for ln in lines if int(ln.split()[0]) == int(ins[0][0]) + 1]
    assert nxt and nxt[0][2] == "mx2"
