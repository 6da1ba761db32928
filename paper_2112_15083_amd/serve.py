"""Continuous-batching request loop over librqc.

Requests (a circuit, an open batch of 2^u amplitudes, optionally rejection
samples) flow through three stages that overlap:

  plan     host worker threads build each request's plan (the C++ planner runs
           outside the GIL); requests whose plan exceeds the cost cap are refused;
  admit    a planned request starts as soon as a stream slot is free and the
           plans in flight plus its own workspace fit the HBM budget; requests
           that can never fit are refused;
  execute  each admitted request runs on its own HIP stream (contraction of its
           batches, then sampling); completion is polled with events, results are
           copied out and the request's workspace is released.

Every request's arithmetic is fixed by its plan (deterministic path search,
fixed kernels and FP64 slice order), so its result does not depend on what
else is in flight.
"""
from __future__ import annotations

import hashlib
import math
import queue
import threading
import time
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
    stream: object = None
    event: object = None
    out: object = None
    samples: object = None
    n_out: int = 0


class Server:
    """One GPU; `n_streams` concurrent requests; HBM admission budget in bytes."""

    def __init__(self, hbm_budget: int | None = None, n_streams: int = 4, plan_workers: int = 4,
                 plan_flops_cap: float = 1e15, plan_opts: dict | None = None, device: int = 0):
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
        self.streams = [torch.cuda.Stream(device=device) for _ in range(n_streams)]
        self.free_streams = list(range(n_streams))
        self.planner = ThreadPoolExecutor(max_workers=plan_workers)
        self.ready: queue.Queue = queue.Queue()
        self.waiting: list = []
        self.running: list = []
        self.lock = threading.Lock()
        self.stop = False
        self.stats = dict(submitted=0, completed=0, refused=0, errors=0)
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
    def _plan(self, w: _Work):
        rqc = self.rqc
        try:
            c = rqc.load_circuit(w.req.text)
            w.plan = rqc.plan_create(c, w.req.open_qubits, precision=w.req.precision, **self.plan_opts)
            w.info = rqc.plan_info(w.plan)
            o = len(w.req.open_qubits)
            out_bytes = len(w.req.fixed_bits) * (8 << o) + 8 * w.req.n_samples
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

    def _launch(self, w: _Work, sid: int):
        rqc, torch = self.rqc, self.torch
        req = w.req
        s = self.streams[sid]
        w.stream = sid
        w.started = time.perf_counter()
        o = len(req.open_qubits)
        with torch.cuda.stream(s):
            w.out = torch.empty((len(req.fixed_bits), 1 << o, 2), dtype=torch.float32, device="cuda")
            rqc.contract_amplitudes(w.plan, req.fixed_bits, w.out, stream=s)
            w.event = torch.cuda.Event()
            w.event.record(s)

    def _complete(self, w: _Work):
        rqc, torch = self.rqc, self.torch
        req = w.req
        s = self.streams[w.stream]
        try:
            if req.n_samples > 0:
                samples = torch.zeros(req.n_samples, dtype=torch.int64, device="cuda")
                n_out, st, _ = rqc.rejection_sample(w.out, req.fixed_bits, req.open_qubits, req.n_qubits,
                                                    req.n_samples, samples, alpha=req.alpha, F_norm=1.0,
                                                    seed=req.seed, stream=s)
                w.samples = samples.cpu().numpy()[:n_out]
                w.n_out = n_out
            torch.cuda.current_stream().wait_stream(s)
            a = w.out.cpu().numpy()
            amps = a[..., 0] + 1j * a[..., 1]
            self._finish(w, "ok", amps=amps)
        except Exception as e:
            self._finish(w, "error", str(e))

    def _finish(self, w: _Work, status: str, msg: str = "", amps=None):
        now = time.perf_counter()
        r = Result(w.req.rid, status, amps=amps, samples=w.samples, n_samples=w.n_out,
                   latency=now - w.req.arrival, queue_wait=(w.started - w.req.arrival) if w.started else 0.0,
                   flops=w.info.get("flops_per_batch", 0.0) * len(w.req.fixed_bits), footprint=w.footprint,
                   message=msg)
        with self.lock:
            key = {"ok": "completed", "refused": "refused", "error": "errors"}[status]
            self.stats[key] += 1
        w.plan = None
        w.out = None
        w.fut.set_result(r)

    def _run(self):
        while not self.stop or self.waiting or self.running or not self.ready.empty():
            progressed = False
            while True:
                try:
                    self.waiting.append(self.ready.get_nowait())
                except queue.Empty:
                    break
            # admission in arrival order among planned requests
            self.waiting.sort(key=lambda x: x.req.arrival)
            still = []
            for w in self.waiting:
                if self.free_streams and self.in_use + w.footprint <= self.budget:
                    sid = self.free_streams.pop(0)
                    self.in_use += w.footprint
                    self.peak_in_use = max(self.peak_in_use, self.in_use)
                    try:
                        self._launch(w, sid)
                        self.running.append(w)
                    except Exception as e:
                        self.in_use -= w.footprint
                        self.free_streams.append(sid)
                        self._finish(w, "error", str(e))
                    progressed = True
                else:
                    still.append(w)
            self.waiting = still
            # completions
            done = [w for w in self.running if w.event.query()]
            for w in done:
                self.running.remove(w)
                self._complete(w)
                self.in_use -= w.footprint
                self.free_streams.append(w.stream)
                progressed = True
            if not progressed:
                time.sleep(0.0002)


def synthetic_requests(n: int, seed: int = 0, shapes=((4, 5), (4, 6), (5, 5), (5, 6)), cycles=(8, 14),
                       log2_amps=(6, 12), sample_frac: float = 0.5, samples=(1000, 4000), bf16_frac: float = 0.5,
                       rate: float | None = None):
    """Seeded request mix: grid shape, depth, 2^u amplitudes, optional samples,
    precision; Poisson arrival offsets when `rate` (requests/s) is given."""
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
        # sampling requests use batches of at least 2^10 amplitudes (16 sub-batches)
        ns = int(rng.integers(samples[0], samples[1] + 1)) if rng.random() < sample_frac and u >= 10 else 0
        n_batches = 1 if ns == 0 else max(1, math.ceil(2.0 * ns / (1 << (u - 6))))
        fixed = synthetic.fixed_bits_batch(nq, open_q, 20_000 + 1000 * rid, n_batches)
        prec = 1 if rng.random() < bf16_frac else 0
        if rate:
            t += float(rng.exponential(1.0 / rate))
        out.append((t, Request(rid, text, nq, open_q, fixed, n_samples=ns, precision=prec)))
    return out


def digest(a: np.ndarray | None) -> str:
    return "" if a is None else hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()[:16]
