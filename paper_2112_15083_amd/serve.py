"""Continuous-batching request loop over librqc.

Requests (a circuit, an open batch of 2^u amplitudes, optionally rejection
samples) flow through three stages that overlap:

  plan     host worker threads build each request's plan (the C++ planner runs
           outside the GIL); the contraction tree and sliced legs depend only on
           the circuit's structure (which gates act where, not which single-qubit
           gate), so they are searched once per structure and kept in a plan
           cache; requests whose plan exceeds the cost cap are refused;
  admit    a planned request is admitted as soon as the plans in flight plus its
           own workspace fit the HBM budget; requests that can never fit are
           refused;
  execute  work units are (request, range of slice groups): a unit adds the
           FP64 sums of its slice groups for all of the request's batches into
           the request's accumulator (rqc_contract_groups).  Each free stream
           takes the next unit of the earliest-arrived admitted request that has
           none in flight (a request's units run one after another: they share
           its plan's workspace), so a long request gives way to others between
           units instead of holding a stream for its whole duration.  After its
           last unit a request is normalised (rqc_finalize_amplitudes), copied
           out and, if it asked for samples, sampled; a sampling request that
           accepted fewer samples than it asked for contracts further batches
           (drawn by the request) and samples them with the next sub-batch
           indices, until it has its count.

A request's units are fixed by its plan (a range size from the planner's time
estimate), and consecutive units carry the FP64 running sum in the
accumulator, so every result is bit-identical to one whole contraction call
and does not depend on what else is in flight.
"""
from __future__ import annotations

import hashlib
import math
import queue
import threading
import time
from collections import OrderedDict
from concurrent.futures import Future, ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    text: str                 # circuit text
    n_qubits: int
    open_qubits: list         # bit b of the batch index = qubit open_qubits[b]
    fixed_bits: list          # one mask per batch
    n_samples: int = 0        # 0 = amplitudes only
    alpha: float = 2.0
    seed: int = 7
    precision: int = 0        # rqc_precision
    arrival: float = 0.0
    # more fixed-bit masks for sampling beyond fixed_bits: (start, count) -> list
    more_fixed_bits: object = None


@dataclass
class Result:
    rid: int
    status: str               # "ok", "refused", "error"
    amps: np.ndarray | None = None
    samples: np.ndarray | None = None
    n_samples: int = 0
    latency: float = 0.0
    queue_wait: float = 0.0
    flops: float = 0.0
    footprint: int = 0
    message: str = ""


@dataclass
class _Work:
    req: Request
    fut: Future
    plan: object = None
    info: dict = field(default_factory=dict)
    footprint: int = 0
    planned_at: float = 0.0
    started: float = 0.0
    stream: object = None     # stream index of the unit in flight (None: no unit in flight)
    event: object = None
    out: object = None
    acc: object = None        # FP64 accumulator of the round's batches
    amps: object = None       # host copy of the requested batches' amplitudes
    cur_fixed: list = field(default_factory=list)  # batches of the round in flight
    cursor: int = 0           # next slice group of the round
    unit: int = 1             # slice groups per work unit
    units_run: int = 0
    sub_done: int = 0         # sub-batches of 64 already sampled
    batches_done: int = 0     # batches contracted so far (all rounds)
    rounds: int = 0
    samples: object = None
    n_out: int = 0


class Server:
    """One GPU; `n_streams` concurrent requests; HBM admission budget in bytes."""

    def __init__(self, hbm_budget: int | None = None, n_streams: int = 4, plan_workers: int = 4,
                 plan_flops_cap: float = 1e15, plan_opts: dict | None = None, device: int = 0,
                 unit_seconds: float = 0.005):
        import torch
        from . import rqc
        self.rqc = rqc
        self.torch = torch
        torch.cuda.set_device(device)
        if hbm_budget is None:
            free, _ = torch.cuda.mem_get_info(device)
            hbm_budget = int(0.9 * free)
        self.budget = int(hbm_budget)
        self.in_use = 0
        self.peak_in_use = 0
        self.cap = plan_flops_cap
        self.plan_opts = dict(n_sliced_target=-1, max_log2_tensor=26, max_log2_batched=26, path_trials=32)
        if plan_opts:
            self.plan_opts.update(plan_opts)
        # plan workspaces come from torch's caching allocator through the C-ABI
        # allocator callbacks, so freeing a finished request's plan never
        # synchronises the device
        self._blocks = {}
        self._blocks_lock = threading.Lock()

        def _alloc(nbytes, ctx):
            t = torch.empty(int(nbytes), dtype=torch.uint8, device=f"cuda:{device}")
            with self._blocks_lock:
                self._blocks[t.data_ptr()] = t
            return t.data_ptr()

        def _free(ptr, ctx):
            with self._blocks_lock:
                self._blocks.pop(ptr, None)

        self._alloc_cb = rqc.ALLOC_FN(_alloc)
        self._free_cb = rqc.FREE_FN(_free)
        self.plan_opts.update(alloc=self._alloc_cb, free=self._free_cb)
        # structure signature -> (path, sliced legs), least recently used first
        self.plan_cache: "OrderedDict[str, tuple]" = OrderedDict()
        self.plan_cache_cap = 256
        self.plan_cache_lock = threading.Lock()
        self.max_rounds = 16
        # target device time of one work unit (the planner's estimate)
        self.unit_seconds = unit_seconds
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        self.admitted: list = []
        self.planner = ThreadPoolExecutor(max_workers=plan_workers)
        self.ready: queue.Queue = queue.Queue()
        self.waiting: list = []
        self.lock = threading.Lock()
        self.stop = False
        self.stats = dict(submitted=0, completed=0, refused=0, errors=0, short=0, plan_cache_hits=0,
                          extra_rounds=0, units=0)
        self.loop = threading.Thread(target=self._run, daemon=True)
        self.loop.start()

    # -------------------------------------------------------------- public
    def submit(self, req: Request) -> Future:
        fut: Future = Future()
        req.arrival = req.arrival or time.perf_counter()
        w = _Work(req, fut)
        with self.lock:
            self.stats["submitted"] += 1
        self.planner.submit(self._plan, w)
        return fut

    def shutdown(self):
        self.stop = True
        self.loop.join()
        self.planner.shutdown(wait=True)

    # -------------------------------------------------------------- stages
    @staticmethod
    def structure_key(req: Request, precision: int) -> str:
        """The circuit text with the single-qubit gate names erased: two circuits
        with the same key have the same tensor network legs."""
        lines = []
        for line in req.text.splitlines():
            tok = line.split()
            if tok and tok[0] in ("sx", "sy", "sw"):
                tok[0] = "g1"
            lines.append(" ".join(tok))
        return hashlib.sha256(("\n".join(lines) + f"|{req.open_qubits}|{precision}").encode()).hexdigest()

    def _plan_for(self, req: Request):
        """Plan on the cached tree and sliced legs of the request's structure;
        a miss searches once and keeps the result.  Every plan is created from
        (path, sliced legs), so a request's plan does not depend on the cache."""
        rqc = self.rqc
        c = rqc.load_circuit(req.text)
        key = self.structure_key(req, req.precision)
        with self.plan_cache_lock:
            hit = self.plan_cache.get(key)
            if hit is not None:
                self.plan_cache.move_to_end(key)
                self.stats["plan_cache_hits"] += 1
        opts = dict(self.plan_opts)
        if hit is None:
            searched = rqc.plan_create(c, req.open_qubits, precision=req.precision, dry_run=1,
                                       **{k: v for k, v in opts.items() if k not in ("alloc", "free")})
            hit = (rqc.plan_path(searched), rqc.plan_sliced_legs(searched))
            del searched
            with self.plan_cache_lock:
                self.plan_cache[key] = hit
                while len(self.plan_cache) > self.plan_cache_cap:
                    self.plan_cache.popitem(last=False)
        path, legs = hit
        return rqc.plan_create(c, req.open_qubits, path=path, sliced_legs=legs, precision=req.precision, **opts)

    def _plan(self, w: _Work):
        rqc = self.rqc
        try:
            w.plan = self._plan_for(w.req)
            w.info = rqc.plan_info(w.plan)
            o = len(w.req.open_qubits)
            # outputs, the FP64 accumulator and the samples
            out_bytes = len(w.req.fixed_bits) * (24 << o) + 8 * w.req.n_samples
            w.footprint = int(w.info["workspace_bytes"]) + out_bytes
            w.planned_at = time.perf_counter()
            flops = w.info["flops_per_batch"] * len(w.req.fixed_bits)
            if flops > self.cap:
                self._finish(w, "refused", f"plan cost {flops:.3g} flops exceeds the cap {self.cap:.3g}")
                return
            if w.footprint > self.budget:
                self._finish(w, "refused", f"footprint {w.footprint} B exceeds the HBM budget {self.budget} B")
                return
            self.ready.put(w)
        except Exception as e:  # planning failures are reported per request
            self._finish(w, "error", str(e))

    def _begin(self, w: _Work):
        """Admission: the request's buffers, its unit size, its first round."""
        torch = self.torch
        req = w.req
        o = len(req.open_qubits)
        n = len(req.fixed_bits)
        w.started = time.perf_counter()
        w.cur_fixed = list(req.fixed_bits)
        w.out = torch.empty((n, 1 << o, 2), dtype=torch.float32, device="cuda")
        w.acc = torch.empty((n, 1 << o, 2), dtype=torch.float64, device="cuda")
        groups = max(1, int(w.info["n_groups"]))
        per_group = w.info["est_seconds"] * n / groups
        w.unit = max(1, min(groups, int(self.unit_seconds / max(per_group, 1e-12))))
        w.cursor = 0

    def _launch_unit(self, w: _Work, sid: int):
        """The request's next range of slice groups on stream sid; the round's
        last unit also normalises into the output."""
        rqc, torch = self.rqc, self.torch
        s = self.streams[sid]
        w.stream = sid
        groups = int(w.info["n_groups"])
        k = min(w.unit, groups - w.cursor)
        nb = len(w.cur_fixed)
        with torch.cuda.stream(s):
            rqc.contract_groups(w.plan, w.cursor, k, w.cur_fixed, w.acc[:nb], stream=s)
            w.cursor += k
            if w.cursor >= groups:
                rqc.finalize_amplitudes(w.plan, w.acc[:nb], nb, w.out[:nb], stream=s)
            w.event = torch.cuda.Event()
            w.event.record(s)
        w.units_run += 1
        with self.lock:
            self.stats["units"] += 1

    def _round_done(self, w: _Work) -> bool:
        """After the round's last unit: copy out, sample.  Returns False when
        another round (more batches for the samples) was started."""
        rqc, torch = self.rqc, self.torch
        req = w.req
        s = self.streams[w.stream]
        try:
            o = len(req.open_qubits)
            if w.rounds == 0:
                torch.cuda.current_stream().wait_stream(s)
                a = w.out.cpu().numpy()
                w.amps = a[..., 0] + 1j * a[..., 1]
            if req.n_samples > 0:
                need = req.n_samples - w.n_out
                with torch.cuda.stream(s):
                    buf = torch.empty(need, dtype=torch.int64, device="cuda")
                    n_out, st, _ = rqc.rejection_sample(w.out[:len(w.cur_fixed)], w.cur_fixed, req.open_qubits,
                                                        req.n_qubits, need, buf, alpha=req.alpha, F_norm=1.0,
                                                        seed=req.seed, batch_index_base=w.sub_done, stream=s)
                got = buf.cpu().numpy()[:n_out]
                w.samples = got if w.samples is None else np.concatenate([w.samples, got])
                w.n_out += n_out
                w.sub_done += len(w.cur_fixed) << (o - 6)
                w.batches_done += len(w.cur_fixed)
                if w.n_out < req.n_samples and req.more_fixed_bits is not None and w.rounds < self.max_rounds:
                    # expected yield about 1/alpha sample per sub-batch; at most
                    # as many batches as the request's own buffers hold
                    want = math.ceil(req.alpha * (req.n_samples - w.n_out) * 1.25 / (1 << (o - 6)))
                    k = max(1, min(len(req.fixed_bits), want))
                    w.cur_fixed = list(req.more_fixed_bits(w.batches_done, k))
                    w.cursor = 0
                    w.rounds += 1
                    with self.lock:
                        self.stats["extra_rounds"] += 1
                    return False
            status = "ok" if w.n_out >= req.n_samples else "short"
            self._finish(w, status, amps=w.amps,
                         msg="" if status == "ok" else f"{w.n_out} of {req.n_samples} samples")
        except Exception as e:
            self._finish(w, "error", str(e))
        return True

    def _finish(self, w: _Work, status: str, msg: str = "", amps=None):
        now = time.perf_counter()
        r = Result(w.req.rid, status, amps=amps, samples=w.samples, n_samples=w.n_out,
                   latency=now - w.req.arrival, queue_wait=(w.started - w.req.arrival) if w.started else 0.0,
                   flops=w.info.get("flops_per_batch", 0.0) * len(w.req.fixed_bits), footprint=w.footprint,
                   message=msg)
        with self.lock:
            key = {"ok": "completed", "refused": "refused", "error": "errors", "short": "short"}[status]
            self.stats[key] += 1
        w.plan = None
        w.out = None
        w.acc = None
        w.fut.set_result(r)

    def _run(self):
        while not self.stop or self.waiting or self.admitted or not self.ready.empty():
            progressed = False
            while True:
                try:
                    self.waiting.append(self.ready.get_nowait())
                except queue.Empty:
                    break
            # admission in arrival order among planned requests, by HBM footprint
            self.waiting.sort(key=lambda x: x.req.arrival)
            still = []
            for w in self.waiting:
                if self.in_use + w.footprint <= self.budget:
                    self.in_use += w.footprint
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    try:
                        self._begin(w)
                        self.admitted.append(w)
                    except Exception as e:
                        self.in_use -= w.footprint
                        self._finish(w, "error", str(e))
                    progressed = True
                else:
                    still.append(w)
            self.waiting = still
            # completed units
            for w in [x for x in self.admitted if x.stream is not None and x.event.query()]:
                progressed = True
                sid = w.stream
                if w.cursor >= int(w.info["n_groups"]):
                    if self._round_done(w):
                        self.admitted.remove(w)
                        self.in_use -= w.footprint
                w.stream = None
                self.free_streams.append(sid)
            # each free stream takes the next unit of the earliest admitted
            # request without a unit in flight
            idle = sorted((x for x in self.admitted if x.stream is None), key=lambda x: x.req.arrival)
            while self.free_streams and idle:
                w = idle.pop(0)
                sid = self.free_streams.pop(0)
                try:
                    self._launch_unit(w, sid)
                except Exception as e:
                    w.stream = None
                    self.free_streams.append(sid)
                    self.admitted.remove(w)
                    self.in_use -= w.footprint
                    self._finish(w, "error", str(e))
                progressed = True
            if not progressed:
                time.sleep(0.0002)


class _MoreFixedBits:
    """Further seeded fixed-bit masks of a synthetic request (batch index i
    draws from seed base + i)."""

    def __init__(self, n_qubits, open_qubits, base):
        self.n, self.open_q, self.base = n_qubits, list(open_qubits), base

    def __call__(self, start, count):
        import synthetic
        return synthetic.fixed_bits_batch(self.n, self.open_q, self.base + start, count)


def synthetic_requests(n: int, seed: int = 0, shapes=((4, 5), (4, 6), (5, 5), (5, 6)), cycles=(8, 14),
                       log2_amps=(6, 12), sample_frac: float = 0.5, samples=(1000, 4000), bf16_frac: float = 0.5,
                       rate: float | None = None, min_log2_for_samples: int = 10):
    """Seeded request mix: grid shape, depth, 2^u amplitudes, optional samples,
    precision; Poisson arrival offsets when `rate` (requests/s) is given.
    Sampling requests get about alpha = 2 sub-batches of 64 per sample, in
    batches of at least 2^min_log2_for_samples amplitudes, and draw more
    masks (seeded) if that does not yield their count."""
    import synthetic
    rng = np.random.default_rng(seed)
    out = []
    t = 0.0
    for rid in range(n):
        r, c = shapes[rng.integers(len(shapes))]
        m = int(rng.integers(cycles[0], cycles[1] + 1))
        nq = r * c
        u = int(rng.integers(log2_amps[0], log2_amps[1] + 1))
        u = min(u, nq)
        open_q = list(range(nq - u, nq))
        text = synthetic.circuit_text(r, c, m, 10_000 + rid)
        ns = int(rng.integers(samples[0], samples[1] + 1)) if rng.random() < sample_frac else 0
        if ns:
            u = max(u, min(min_log2_for_samples, nq))
            open_q = list(range(nq - u, nq))
        n_batches = 1 if ns == 0 else max(1, math.ceil(2.0 * ns / (1 << (u - 6))))
        fixed = synthetic.fixed_bits_batch(nq, open_q, 20_000 + 1000 * rid, n_batches)
        prec = 1 if rng.random() < bf16_frac else 0
        if rate:
            t += float(rng.exponential(1.0 / rate))
        more = _MoreFixedBits(nq, open_q, 20_000 + 1000 * rid) if ns else None
        out.append((t, Request(rid, text, nq, open_q, fixed, n_samples=ns, precision=prec, more_fixed_bits=more)))
    return out


def digest(a: np.ndarray | None) -> str:
    return "" if a is None else hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]
