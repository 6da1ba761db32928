"""ctypes binding of librqc (include/rqc.h): argument marshalling only.

Every function has the name of its C entry point without the ``rqc_`` prefix.
Device buffers are passed as torch tensors (their data_ptr) or raw integer
addresses; streams as torch.cuda.Stream objects, raw handles, or None for the
current torch stream.  A non-OK status raises RqcError carrying the library's
message.  The library must be built (python -m paper_2112_15083_amd.build);
importing this module without it raises ImportError.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librqc.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"librqc.so is not built ({LIB_PATH}); run python -m paper_2112_15083_amd.build")

# One HIP runtime per process: PyTorch ships its own libamdhip64 (soname
# libamdhip64.so.7).  Loaded first, it satisfies librqc's dependency of that
# soname, so the streams and device pointers torch hands over belong to the
# runtime the library calls.  Loaded after librqc, it would come in as a second
# runtime beside the system one, and one of the two would find no device.
try:
    import torch  # noqa: F401
except ImportError:  # the library itself does not need torch
    pass

_lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, EPARSE, EPLAN, ENOMEM, EDEVICE, ESHORT = 0, -1, -2, -3, -4, -5, -6
C64, BF16X3, FP16X3 = 0, 1, 2
K_LEAF, K_SMALL, K_STREAM, K_PERMUTE, K_GEMM, K_ACCUM, K_FINAL, K_SAMPLE = range(8)
K_NAMES = ["leaf_select", "small_trees", "stream", "permute", "gemm", "accumulate", "finalize", "sample"]

# rqc_plan_info_t.stream_kernels entries
STREAM_KERNELS = ["mx2", "mx", "lk", "ky", "tile", "gen"]

ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class PlanOpts(ctypes.Structure):
    _fields_ = [("max_log2_tensor", ctypes.c_int32), ("n_sliced_target", ctypes.c_int32),
                ("max_log2_batched", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("target_fidelity", ctypes.c_double), ("partial_k", ctypes.c_int32),
                ("partial_count", ctypes.c_int32), ("partial_total_slices", ctypes.c_int64),
                ("path_trials", ctypes.c_int32),
                ("path_seed", ctypes.c_uint64), ("profile", ctypes.c_int32), ("dry_run", ctypes.c_int32),
                ("alloc", ALLOC_FN), ("free", FREE_FN), ("alloc_ctx", ctypes.c_void_p),
                ("global_cache", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("no_stream_fusion", ctypes.c_int32), ("no_matrix_core_streams", ctypes.c_int32),
                ("anneal_iters", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_qubits", ctypes.c_int32), ("n_open", ctypes.c_int32), ("n_variables", ctypes.c_int32),
                ("n_sliced", ctypes.c_int32), ("n_batched", ctypes.c_int32), ("n_partial", ctypes.c_int32),
                ("n_slices", ctypes.c_int64), ("n_partial_kept", ctypes.c_int64), ("fidelity", ctypes.c_double),
                ("flops_per_batch", ctypes.c_double), ("flops_unsliced", ctypes.c_double),
                ("gemm_flop_share", ctypes.c_double), ("bytes_per_batch", ctypes.c_double),
                ("max_log2_tensor", ctypes.c_int32), ("n_steps", ctypes.c_int32),
                ("n_launches", ctypes.c_int32), ("n_groups", ctypes.c_int64),
                ("workspace_bytes", ctypes.c_int64), ("plan_seconds", ctypes.c_double),
                ("cache_bytes", ctypes.c_int64), ("flops_cached", ctypes.c_double),
                ("est_seconds", ctypes.c_double), ("n_fused", ctypes.c_int32),
                ("stream_kernels", ctypes.c_int32 * 8)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["stream_kernels"] = dict(zip(STREAM_KERNELS, list(self.stream_kernels)))
        return d


class SampleStats(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int64), ("batches", ctypes.c_int64), ("batches_used", ctypes.c_int64),
                ("eps_J", ctypes.c_double), ("p_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Profile(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64 * 8), ("seconds", ctypes.c_double * 8),
                ("flops", ctypes.c_double * 8), ("bytes", ctypes.c_double * 8)]

    def as_dict(self):
        return {K_NAMES[i]: dict(launches=self.launches[i], seconds=self.seconds[i], flops=self.flops[i],
                                 bytes=self.bytes[i]) for i in range(8)}


class OpProfile(ctypes.Structure):
    _fields_ = [("cls", ctypes.c_int32), ("op", ctypes.c_int32), ("launches", ctypes.c_int64),
                ("seconds", ctypes.c_double), ("flops", ctypes.c_double), ("bytes", ctypes.c_double),
                ("exec_flops", ctypes.c_double), ("exec_kind", ctypes.c_int32), ("pad", ctypes.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "pad"}
        d["cls"] = K_NAMES[self.cls]
        return d


_P = ctypes.c_void_p
_sig = {
    "rqc_load_circuit": [ctypes.c_char_p, ctypes.c_size_t, ctypes.POINTER(_P)],
    "rqc_circuit_info": [_P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32)],
    "rqc_plan_create": [_P, _P, ctypes.c_int32, _P, ctypes.c_int32, _P, ctypes.c_int32,
                        ctypes.POINTER(PlanOpts), ctypes.POINTER(_P)],
    "rqc_plan_info": [_P, ctypes.POINTER(PlanInfo)],
    "rqc_plan_sliced_legs": [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "rqc_plan_path": [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "rqc_plan_describe": [_P, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)],
    "rqc_plan_partial": [_P, _P, ctypes.c_int32, _P, ctypes.c_int64, _P, ctypes.c_int64],
    "rqc_plan_slices": [_P, _P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)],
    "rqc_plan_profile": [_P, ctypes.POINTER(Profile)],
    "rqc_plan_profile_reset": [_P],
    "rqc_plan_profile_classes": [_P, ctypes.c_uint32],
    "rqc_plan_profile_ops": [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "rqc_contract_amplitudes": [_P, _P, ctypes.c_int64, _P, ctypes.c_int64, _P, _P, _P],
    "rqc_contract_groups": [_P, ctypes.c_int64, ctypes.c_int64, _P, ctypes.c_int64, _P, _P],
    "rqc_finalize_amplitudes": [_P, _P, ctypes.c_int64, _P, _P, _P],
    "rqc_kernel_cgemm": [_P, _P, _P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "rqc_kernel_permute": [_P, _P, ctypes.c_int32, _P, _P],
    "rqc_rejection_sample": [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                             ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                             ctypes.c_int64, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64),
                             ctypes.POINTER(SampleStats), _P],
    "rqc_select_top": [_P, ctypes.c_uint64, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int64, _P, _P],
    "rqc_prob_sums": [_P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, _P, _P, _P],
    "rqc_rejection_sample_static": [_P, _P, ctypes.c_int64, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_uint64, ctypes.c_uint64,
                                    ctypes.c_int64, ctypes.c_int64, _P, ctypes.POINTER(ctypes.c_int64),
                                    ctypes.POINTER(SampleStats), _P],
}
for _name, _args in _sig.items():
    _f = getattr(_lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
_lib.rqc_last_error.restype = ctypes.c_char_p
_lib.rqc_version.restype = ctypes.c_char_p
_lib.rqc_plan_destroy.argtypes = [_P]
_lib.rqc_plan_destroy.restype = None
_lib.rqc_circuit_destroy.argtypes = [_P]
_lib.rqc_circuit_destroy.restype = None

EXPORTS = sorted(list(_sig) + ["rqc_last_error", "rqc_version", "rqc_plan_destroy", "rqc_circuit_destroy"])


class RqcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"librqc status {status}: {msg}")
        self.status = status


def last_error() -> str:
    return _lib.rqc_last_error().decode()


def version() -> str:
    return _lib.rqc_version().decode()


def _check(st, allow=()):
    if st != OK and st not in allow:
        raise RqcError(st, last_error())
    return st


def _ptr(x):
    """Device/host address of a torch tensor, numpy array, int or None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def _stream(s):
    if s is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(s, int):
        return s
    return s.cuda_stream


def _i32(seq):
    arr = (ctypes.c_int32 * max(1, len(seq)))(*seq)
    return arr


def _u64(seq):
    return (ctypes.c_uint64 * max(1, len(seq)))(*[int(v) & (2 ** 64 - 1) for v in seq])


class Circuit:
    def __init__(self, handle):
        self.handle = handle

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rqc_circuit_destroy(self.handle)
            self.handle = None


class Plan:
    def __init__(self, handle, open_qubits):
        self.handle = handle
        self.open_qubits = list(open_qubits)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.rqc_plan_destroy(self.handle)
            self.handle = None


def load_circuit(text: str) -> Circuit:
    b = text.encode()
    h = _P()
    _check(_lib.rqc_load_circuit(b, len(b), ctypes.byref(h)))
    return Circuit(h)


def circuit_info(c: Circuit):
    n, v, g = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(_lib.rqc_circuit_info(c.handle, ctypes.byref(n), ctypes.byref(v), ctypes.byref(g)))
    return dict(n_qubits=n.value, n_variables=v.value, n_gates=g.value)


def make_opts(**kw) -> PlanOpts:
    o = PlanOpts()
    for k, v in kw.items():
        if v is not None:
            setattr(o, k, v)
    return o


def plan_create(c: Circuit, open_qubits, path=None, sliced_legs=None, opts: PlanOpts | None = None,
                **kw) -> Plan:
    if opts is None:
        opts = make_opts(**kw)
    flat = [x for pr in path for x in pr] if path is not None else None
    h = _P()
    _check(_lib.rqc_plan_create(c.handle, _i32(flat) if flat is not None else None,
                                len(path) if path is not None else 0,
                                _i32(sliced_legs) if sliced_legs is not None else None,
                                len(sliced_legs) if sliced_legs is not None else 0,
                                _i32(list(open_qubits)), len(open_qubits), ctypes.byref(opts), ctypes.byref(h)))
    return Plan(h, open_qubits)


def plan_info(p: Plan) -> dict:
    info = PlanInfo()
    _check(_lib.rqc_plan_info(p.handle, ctypes.byref(info)))
    return info.as_dict()


def plan_describe(p: Plan) -> str:
    """The plan's launch program, one op per line (see rqc_plan_describe)."""
    n = ctypes.c_size_t()
    _check(_lib.rqc_plan_describe(p.handle, None, 0, ctypes.byref(n)))
    buf = ctypes.create_string_buffer(n.value)
    _check(_lib.rqc_plan_describe(p.handle, buf, n.value, ctypes.byref(n)))
    return buf.value.decode()


def plan_sliced_legs(p: Plan):
    n = ctypes.c_int32()
    _check(_lib.rqc_plan_sliced_legs(p.handle, None, 0, ctypes.byref(n)))
    arr = (ctypes.c_int32 * max(1, n.value))()
    _check(_lib.rqc_plan_sliced_legs(p.handle, arr, n.value, ctypes.byref(n)))
    return list(arr)[: n.value]


def plan_path(p: Plan):
    """The plan's contraction tree as SSA pairs (the `path` plan_create takes)."""
    n = ctypes.c_int32()
    _check(_lib.rqc_plan_path(p.handle, None, 0, ctypes.byref(n)))
    arr = (ctypes.c_int32 * max(2, 2 * n.value))()
    _check(_lib.rqc_plan_path(p.handle, arr, n.value, ctypes.byref(n)))
    return [(arr[2 * s], arr[2 * s + 1]) for s in range(n.value)]


def plan_partial(p: Plan):
    info = plan_info(p)
    k, nx = info["n_partial"], info["n_partial_kept"]
    S = (ctypes.c_int32 * max(1, k))()
    X = (ctypes.c_uint64 * max(1, nx))()
    nr = (1 << k) if k and nx else 0  # a host-only plan selects S but has no norms
    R = (ctypes.c_double * max(1, nr))()
    _check(_lib.rqc_plan_partial(p.handle, S, k, X, nx, R, nr))
    return list(S)[:k], list(X)[:nx], list(R)[:nr]


def plan_slices(p: Plan, cap: int | None = None):
    """The plan's default slice list (slice ids), at most `cap` of them."""
    n = ctypes.c_int64()
    _check(_lib.rqc_plan_slices(p.handle, None, 0, ctypes.byref(n)))
    k = n.value if cap is None else min(cap, n.value)
    arr = (ctypes.c_uint64 * max(1, k))()
    _check(_lib.rqc_plan_slices(p.handle, arr, k, ctypes.byref(n)))
    return list(arr)[:k]


def plan_profile(p: Plan) -> dict:
    pr = Profile()
    _check(_lib.rqc_plan_profile(p.handle, ctypes.byref(pr)))
    return pr.as_dict()


def plan_profile_ops(p: Plan) -> list:
    """Per-op profile records (see rqc_op_profile_t)."""
    n = ctypes.c_int32()
    _check(_lib.rqc_plan_profile_ops(p.handle, None, 0, ctypes.byref(n)))
    arr = (OpProfile * max(1, n.value))()
    _check(_lib.rqc_plan_profile_ops(p.handle, arr, n.value, ctypes.byref(n)))
    return [arr[i].as_dict() for i in range(n.value)]


def plan_profile_reset(p: Plan):
    _check(_lib.rqc_plan_profile_reset(p.handle))


def plan_profile_classes(p: Plan, classes):
    """Time only the launches of these classes (names as in K_NAMES)."""
    mask = 0
    for c in classes:
        mask |= 1 << K_NAMES.index(c)
    _check(_lib.rqc_plan_profile_classes(p.handle, mask))


def contract_amplitudes(p: Plan, fixed_bits, out_amps, out_f64=None, slice_ids=None, stream=None):
    fb = _u64(list(fixed_bits))
    sl = _u64(list(slice_ids)) if slice_ids is not None else None
    _check(_lib.rqc_contract_amplitudes(p.handle, sl, len(slice_ids) if slice_ids is not None else 0, fb,
                                        len(fixed_bits), _ptr(out_amps), _ptr(out_f64), _stream(stream)))


def contract_groups(p: Plan, first_group, n_groups, fixed_bits, acc_f64, stream=None):
    """Add the FP64 sums of default slice groups [first_group, first_group +
    n_groups) into acc_f64 (complex128 [n_batches][2^o]; overwritten when
    first_group is 0).  Asynchronous."""
    _check(_lib.rqc_contract_groups(p.handle, first_group, n_groups, _u64(list(fixed_bits)), len(fixed_bits),
                                    _ptr(acc_f64), _stream(stream)))


def finalize_amplitudes(p: Plan, acc_f64, n_batches, out_amps, out_f64=None, stream=None):
    """Normalised complex64 (and optional FP64) amplitudes from an accumulator
    filled by contract_groups.  Asynchronous."""
    _check(_lib.rqc_finalize_amplitudes(p.handle, _ptr(acc_f64), n_batches, _ptr(out_amps), _ptr(out_f64),
                                        _stream(stream)))


def rejection_sample(amps, fixed_bits, open_qubits, n_qubits, n_samples, out_samples, alpha=2.0, F_norm=1.0,
                     seed=7, batch_index_base=0, log2_NA=6, pick_steps=0, stream=None):
    """Returns (n_out, stats dict, status) -- status is OK or ESHORT."""
    n_out = ctypes.c_int64()
    st = SampleStats()
    code = _check(_lib.rqc_rejection_sample(_ptr(amps), _u64(list(fixed_bits)), len(fixed_bits),
                                            _i32(list(open_qubits)), len(open_qubits), log2_NA, n_qubits,
                                            alpha, F_norm, seed, batch_index_base, pick_steps, n_samples,
                                            _ptr(out_samples), ctypes.byref(n_out), ctypes.byref(st),
                                            _stream(stream)), allow=(ESHORT,))
    return n_out.value, st.as_dict(), code


def rejection_sample_static(amps, fixed_bits, open_qubits, n_qubits, n_samples, out_samples, alpha=2.0,
                            F_norm=1.0, seed=7, batch_index_base=0, log2_NA=6, pick_steps=0, stream=None):
    """rejection_sample with its scratch in the library's fixed device array
    (no allocation).  Returns (n_out, stats dict, status)."""
    n_out = ctypes.c_int64()
    st = SampleStats()
    code = _check(_lib.rqc_rejection_sample_static(_ptr(amps), _u64(list(fixed_bits)), len(fixed_bits),
                                                   _i32(list(open_qubits)), len(open_qubits), log2_NA, n_qubits,
                                                   alpha, F_norm, seed, batch_index_base, pick_steps, n_samples,
                                                   _ptr(out_samples), ctypes.byref(n_out), ctypes.byref(st),
                                                   _stream(stream)), allow=(ESHORT,))
    return n_out.value, st.as_dict(), code


SAMPLE_STATIC_SCRATCH_BYTES = 8 << 20  # RQC_SAMPLE_STATIC_SCRATCH_BYTES


def select_top(amps, fixed_bits, open_qubits, n_qubits, count, out_samples, stream=None):
    """The `count` bitstrings of one batch with the largest |amplitude|^2, in
    ascending batch index (asynchronous)."""
    _check(_lib.rqc_select_top(_ptr(amps), int(fixed_bits) & (2 ** 64 - 1), _i32(list(open_qubits)),
                               len(open_qubits), n_qubits, count, _ptr(out_samples), _stream(stream)))


def prob_sums(amps, n_rows, row_len, n_qubits, sums, xeb=None, stream=None):
    """FP64 sums of |a|^2 over each of n_rows rows of row_len amplitudes, and
    the linear XEB 2^n * sum / row_len - 1 of each row into `xeb` when given
    (asynchronous)."""
    _check(_lib.rqc_prob_sums(_ptr(amps), n_rows, row_len, n_qubits, _ptr(sums), _ptr(xeb), _stream(stream)))


def kernel_cgemm(A, B, C, batch, M, N, K, a_kfast=1, b_nfast=1, precision=C64, stream=None):
    _check(_lib.rqc_kernel_cgemm(_ptr(A), _ptr(B), _ptr(C), batch, M, N, K, a_kfast, b_nfast, precision,
                                 _stream(stream)))


def kernel_permute(src, dst, perm, stream=None):
    _check(_lib.rqc_kernel_permute(_ptr(src), _ptr(dst), len(perm), _i32(list(perm)), _stream(stream)))


def plan_destroy(p: Plan):
    if p.handle:
        _lib.rqc_plan_destroy(p.handle)
        p.handle = None


def circuit_destroy(c: Circuit):
    if c.handle:
        _lib.rqc_circuit_destroy(c.handle)
        c.handle = None
