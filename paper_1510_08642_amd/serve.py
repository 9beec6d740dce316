"""Continuous-batching request loop for DD products and DD LU solves.

Requests (a DD product C = A B, or a factor-then-solve A X = B) arrive over
time.  The loop admits the oldest waiting request as soon as a slot (a HIP
stream) and enough of the device-memory budget are free; small products that
are waiting together are merged into one grouped launch; admitted work on
different slots overlaps on the GPU.  Completion is read from events, memory
is returned to the budget, and the next requests are admitted while others are
still running.  Factorisations can be kept resident (``factorize`` /
``solve``) for later right-hand sides.

The scheduling logic is independent of the device: it drives an *executor*
(``GpuExecutor`` here; tests substitute a CPU one), so admission, batching and
back-pressure are testable without a GPU.  No request's arithmetic depends on
what it is batched with: the grouped launch computes each product exactly as a
single Block product would.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Any, Callable, Optional

import numpy as np


@dataclasses.dataclass
class Request:
    rid: int
    kind: str                  # "gemm" or "lu"
    n: int
    nrhs: int = 0
    t_arrive: float = 0.0      # seconds from the start of the run
    payload: Any = None        # executor-specific inputs
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    result: Any = None
    error: Optional[str] = None
    batch_size: int = 1
    bypassed: int = 0          # later requests admitted while this one was the head

    @property
    def latency(self) -> Optional[float]:
        if self.t_done is None:
            return None
        return self.t_done - self.t_arrive


@dataclasses.dataclass
class Stats:
    completed: int
    failed: int
    wall_s: float
    p50_ms: float
    p99_ms: float
    mean_ms: float
    throughput_rps: float
    gflops: float
    batches: int
    max_inflight_bytes: int

    def as_dict(self):
        return dataclasses.asdict(self)


def request_flops(r: Request) -> float:
    """Effective flops: 2 n^3 for a product, 2/3 n^3 + 2 n^2 nrhs for a solve."""
    if r.kind == "gemm":
        return 2.0 * r.n ** 3
    return 2.0 / 3.0 * r.n ** 3 + 2.0 * r.n ** 2 * r.nrhs


class Server:
    """Admission by memory footprint, oldest first, continuous batching.

    budget_bytes  device memory the in-flight requests may use together
    slots         concurrent launch streams
    small_n       products with n <= small_n are merged into grouped launches
    max_batch     at most this many products per grouped launch
    reserve_small slots kept for small requests (work <= small_flops): large
                  requests start only while more slots than this are free, so
                  a burst of large factorizations cannot hold every slot
    max_bypass    a head that does not fit (memory, or a slot held back for
                  small requests) lets later requests that fit go first, at
                  most this many times; then it waits alone (no starvation)
    window        how far behind the head admission looks for such requests
    """

    def __init__(self, executor, budget_bytes: int, slots: int = 4, small_n: int = 256,
                 max_batch: int = 24, poll_sleep_s: float = 0.0, reserve_small: int = 0,
                 small_flops: float = 2.0 * 512 ** 3, max_bypass: int = 32, window: int = 64):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.small_n = small_n
        self.max_batch = max_batch
        self.poll_sleep_s = poll_sleep_s
        self.reserve_small = int(reserve_small)
        self.small_flops = small_flops
        self.max_bypass = max_bypass
        self.window = window

    def _batchable(self, r: Request) -> bool:
        return r.kind == "gemm" and r.n <= self.small_n and self.ex.can_group

    def _small(self, r: Request) -> bool:
        return request_flops(r) <= self.small_flops

    def _fits(self, r: Request, fp: int) -> bool:
        if fp > self._free_bytes:
            return False
        return self._small(r) or len(self._free_slots) > self.reserve_small

    # -- the loop's state and one scheduling pass (shared with OnlineServer) --
    def _reset(self):
        self._queue: collections.deque = collections.deque()
        self._inflight = []                 # (handle, batch, bytes, slot)
        self._free_slots = list(range(self.slots))
        self._free_bytes = self.budget
        self._max_used = 0
        self._batches = 0

    def _step(self, now: float, on_done: Optional[Callable[[list], None]] = None) -> bool:
        """Completes finished batches, then admits waiting requests oldest
        first while a slot and enough of the budget are free.  Returns whether
        anything changed.  on_done(batch) is called for every finished or
        failed request list."""
        progressed = False
        for item in list(self._inflight):
            h, batch, nbytes, slot = item
            if self.ex.done(h):
                t_done = self.ex.finish(h, batch)
                for r in batch:
                    r.t_done = t_done if t_done is not None else now
                self._inflight.remove(item)
                self._free_bytes += nbytes
                self._free_slots.append(slot)
                progressed = True
                if on_done:
                    on_done(batch)
        queue = self._queue
        while queue and self._free_slots:
            head = queue[0]
            fp = self.ex.footprint(head)
            if fp > self.budget:
                queue.popleft()
                head.error = f"footprint {fp} exceeds the budget {self.budget}"
                progressed = True
                if on_done:
                    on_done([head])
                continue
            pick = 0
            if not self._fits(head, fp):
                # back-pressure: the head waits; a later request that fits may
                # go first while the head has been passed fewer than
                # max_bypass times
                pick = -1
                if head.bypassed < self.max_bypass:
                    for k in range(1, min(len(queue), self.window)):
                        f = self.ex.footprint(queue[k])
                        if f <= self.budget and self._fits(queue[k], f):
                            pick, fp = k, f
                            break
                if pick < 0:
                    break
                head.bypassed += 1
            first = queue[pick]
            del queue[pick]
            batch = [first]
            used = fp
            if self._batchable(first):
                keep = collections.deque()
                scanned = 0
                while queue and len(batch) < self.max_batch and scanned < self.window:
                    r = queue.popleft()
                    scanned += 1
                    f = self.ex.footprint(r)
                    if self._batchable(r) and used + f <= self._free_bytes:
                        batch.append(r)
                        used += f
                    else:
                        keep.append(r)
                queue.extendleft(reversed(keep))
            slot = self._free_slots.pop()
            for r in batch:
                r.t_admit = now
                r.batch_size = len(batch)
            try:
                h = self.ex.launch(batch, slot)
            except Exception as exc:           # the batch fails, the loop goes on
                for r in batch:
                    r.error = f"{type(exc).__name__}: {exc}"
                    r.t_done = now
                self._free_slots.append(slot)
                progressed = True
                if on_done:
                    on_done(batch)
                continue
            self._free_bytes -= used
            self._max_used = max(self._max_used, self.budget - self._free_bytes)
            self._inflight.append((h, batch, used, slot))
            self._batches += 1
            progressed = True
        return progressed

    def run(self, requests, clock: Callable[[], float] = time.perf_counter) -> Stats:
        """Replays a trace: each request joins the queue at its t_arrive."""
        reqs = sorted(requests, key=lambda r: r.t_arrive)
        pending = collections.deque(reqs)
        self._reset()
        self.ex.start()
        t0 = clock()
        while pending or self._queue or self._inflight:
            now = clock() - t0
            while pending and pending[0].t_arrive <= now:
                self._queue.append(pending.popleft())
            progressed = self._step(clock() - t0)
            if not progressed:
                if self.poll_sleep_s:
                    time.sleep(self.poll_sleep_s)
                elif not self._inflight and pending and not self._queue:
                    # idle until the next arrival
                    wait = pending[0].t_arrive - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
        wall = clock() - t0
        self.ex.stop()
        return summarize(reqs, wall, self._batches, self._max_used)


def summarize(reqs, wall: float, batches: int, max_used: int) -> Stats:
    done = [r for r in reqs if r.error is None and r.t_done is not None]
    lat = np.array([r.latency for r in done]) * 1e3 if done else np.zeros(1)
    flops = sum(request_flops(r) for r in done)
    return Stats(completed=len(done), failed=len(reqs) - len(done), wall_s=wall,
                 p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                 mean_ms=float(np.mean(lat)), throughput_rps=len(done) / wall if wall else 0.0,
                 gflops=flops / wall / 1e9 if wall else 0.0, batches=batches,
                 max_inflight_bytes=max_used)


class OnlineServer:
    """Live front end of the same loop: requests are submitted from any
    thread and answered through futures, while a scheduler thread admits,
    batches and completes them.

        srv = OnlineServer(GpuExecutor(slots=4), budget_bytes=1 << 30)
        f = srv.submit_gemm(A, B)          # square DD (2, n, n) device tensors
        g = srv.submit_lu_solve(A, B)      # A (2, n, n), B (2, n, nrhs)
        C, X = f.result(), g.result()
        h = srv.factorize(A); X2 = srv.solve(h, B2)   # resident factors
        srv.close()                                   # finishes queued work
    """

    def __init__(self, executor, budget_bytes: int, slots: int = 4, small_n: int = 256,
                 max_batch: int = 24, clock: Callable[[], float] = time.perf_counter,
                 idle_sleep_s: float = 50e-6):
        import concurrent.futures
        import itertools
        import queue
        import threading
        self._Future = concurrent.futures.Future
        self.core = Server(executor, budget_bytes, slots, small_n, max_batch)
        self.ex = executor
        self.clock = clock
        self.idle_sleep_s = idle_sleep_s
        self._in = queue.SimpleQueue()
        self._futs = {}
        self._done_reqs = []
        self._ids = itertools.count()
        self._lock = threading.Lock()
        self._stop = threading.Event()
        self._keys = itertools.count()
        self.core._reset()
        self.ex.start()
        self._t0 = clock()
        self._thread = threading.Thread(target=self._loop, name="ddqd-serve", daemon=True)
        self._thread.start()

    def _submit(self, kind: str, n: int, nrhs: int, payload):
        if self._stop.is_set():
            raise RuntimeError("server is closed")
        fut = self._Future()
        r = Request(rid=next(self._ids), kind=kind, n=n, nrhs=nrhs, payload=payload)
        with self._lock:
            self._futs[r.rid] = (fut, r)
        self._in.put(r)
        return fut

    def submit_gemm(self, A, B):
        """C = A B (DD, square n x n operands); the future's result is C."""
        n = A.shape[1]
        if A.shape[0] != 2 or B.shape[0] != 2 or tuple(A.shape[1:]) != (n, n) or \
                tuple(B.shape[1:]) != (n, n):
            raise ValueError("submit_gemm takes square DD operands of one size")
        return self._submit("gemm", n, 0, (A, B))

    def submit_lu_solve(self, A, B):
        """X = A^-1 B by LU with partial pivoting; the future's result is X."""
        n = A.shape[1]
        if A.shape[0] != 2 or tuple(A.shape[1:]) != (n, n) or B.shape[0] != 2 or \
                B.shape[1] != n:
            raise ValueError("submit_lu_solve takes A (2, n, n) and B (2, n, nrhs)")
        return self._submit("lu", n, B.shape[2], (A, B))

    def factorize(self, A):
        """Factors A and keeps the factors on the device; returns a handle."""
        return self.ex.factorize(A, ("resident", next(self._keys)))

    def solve(self, handle, B):
        return self.ex.solve(handle, B)

    def release(self, handle):
        self.ex.release(handle)

    def stats(self) -> Stats:
        with self._lock:
            reqs = list(self._done_reqs)
        return summarize(reqs, self.clock() - self._t0, self.core._batches, self.core._max_used)

    def close(self, timeout: Optional[float] = None):
        self._stop.set()
        self._thread.join(timeout)
        self.ex.stop()

    def _complete(self, batch):
        with self._lock:
            for r in batch:
                fut, _ = self._futs.pop(r.rid)
                self._done_reqs.append(r)
                r.payload = None
                if r.error is not None:
                    fut.set_exception(RuntimeError(r.error))
                else:
                    fut.set_result(r.result)

    def _loop(self):
        core = self.core
        while True:
            now = self.clock() - self._t0
            got = False
            while True:
                try:
                    r = self._in.get_nowait()
                except Exception:
                    break
                r.t_arrive = now
                core._queue.append(r)
                got = True
            progressed = core._step(self.clock() - self._t0, on_done=self._complete) or got
            if self._stop.is_set() and not core._queue and not core._inflight and \
                    self._in.empty():
                return
            if not progressed:
                time.sleep(self.idle_sleep_s)


class GpuExecutor:
    """Runs requests with the HIP library on one GPU, one stream per slot.

    Small products waiting together are merged into one grouped call on
    either base (FMA: persistent Block launches; Ozaki: one exponent, one
    slicing and one product launch per group), each result bit-identical to
    the product run alone.

    Request inputs are views into device-resident pools (so a request's
    latency is queueing plus device work, not PCIe).  payload of a "gemm"
    request: (A, B) device DD tensors; of an "lu" request: (A, B) with A
    copied before it is factored in place."""

    can_group = True

    def __init__(self, slots: int, base: str = "fma", gemm_algo: str = "block",
                 gemm_levels: int = 0, lu_panel: int = 128, lu_algo: str = "winograd",
                 lu_levels: int = 1, keep_factors: bool = False, device: str = "cuda:0"):
        import torch

        from . import ddqd
        self.torch, self.dd = torch, ddqd
        self.dev = torch.device(device)
        self.streams = [torch.cuda.Stream(self.dev) for _ in range(slots)]
        self.base = base
        self.gemm_algo, self.gemm_levels = gemm_algo, gemm_levels
        self.lu_panel, self.lu_algo, self.lu_levels = lu_panel, lu_algo, lu_levels
        self.keep_factors = keep_factors
        self.factors = {}
        self._t0 = None

    # -- memory accounting -------------------------------------------------
    def footprint(self, r: Request) -> int:
        n = r.n
        if r.kind == "gemm":
            ws = self.dd.gemm_workspace(2, n, n, n, self.gemm_algo if r.n > 256 else "block",
                                        self.gemm_levels if r.n > 256 else 0, self.base)
            return 16 * n * n + ws
        ws = self.dd.getrf_workspace(n, min(self.lu_panel, n), self.lu_algo, self.lu_levels,
                                     self.base)
        return 16 * n * n + 32 * n * r.nrhs + ws + 8 * n + 64 * n * min(r.nrhs, 16) + 4096

    # -- lifecycle ----------------------------------------------------------
    def start(self):
        torch = self.torch
        torch.cuda.synchronize(self.dev)
        self._t0 = torch.cuda.Event(enable_timing=True)
        self._t0.record(torch.cuda.current_stream(self.dev))

    def stop(self):
        self.torch.cuda.synchronize(self.dev)

    def launch(self, batch, slot):
        torch, dd = self.torch, self.dd
        st = self.streams[slot]
        # inputs were produced on the current stream before the run
        st.wait_stream(torch.cuda.current_stream(self.dev))
        outs = []
        with torch.cuda.stream(st):
            if batch[0].kind == "gemm" and len(batch) > 1:
                probs = []
                for r in batch:
                    A, B = r.payload
                    C = torch.empty((2, r.n, r.n), dtype=torch.float64, device=self.dev)
                    probs.append((A, B, C, 1, 0))
                    outs.append(C)
                dd.dd_gemm_grouped(probs, base=self.base)
            elif batch[0].kind == "gemm":
                r = batch[0]
                A, B = r.payload
                small = r.n <= 256
                C = dd.dd_gemm(A, B, algo="block" if small else self.gemm_algo,
                               levels=0 if small else self.gemm_levels, base=self.base)
                outs.append(C)
            else:
                r = batch[0]
                A, B = r.payload
                LU = A.clone()
                X = B.clone()
                ipiv, perm, info = dd.dd_getrf(LU, panel=min(self.lu_panel, r.n),
                                               algo=self.lu_algo, levels=self.lu_levels,
                                               base=self.base)
                dd.dd_getrs(LU, ipiv, X, perm=perm)
                outs.append(X)
                if self.keep_factors:
                    self.factors[r.rid] = (LU, ipiv, perm, info)
            ev = torch.cuda.Event(enable_timing=True)
            ev.record(st)
        return (ev, outs)

    def done(self, h) -> bool:
        return h[0].query()

    def finish(self, h, batch):
        ev, outs = h
        for r, o in zip(batch, outs):
            r.result = o
        return self._t0.elapsed_time(ev) * 1e-3

    # -- resident factorisations -------------------------------------------
    def factorize(self, A, key):
        dd = self.dd
        LU = A.clone()
        ipiv, perm, info = dd.dd_getrf(LU, panel=min(self.lu_panel, A.shape[1]),
                                       algo=self.lu_algo, levels=self.lu_levels, base=self.base)
        self.factors[key] = (LU, ipiv, perm, info)
        return key

    def solve(self, key, B):
        LU, ipiv, perm, _ = self.factors[key]
        X = B.clone()
        self.dd.dd_getrs(LU, ipiv, X, perm=perm)
        return X

    def release(self, key):
        self.factors.pop(key, None)


class DevicePools:
    """Device-resident random DD pools that request inputs are views of.

    gemm: views A[:, o:o+n, p:p+n] of a uniform pool (leading dimension = the
    pool's); lu: leading-diagonal blocks of an N(0, 1) + nmax I pool (so every
    block is diagonally dominant) and uniform right-hand sides."""

    def __init__(self, nmax_gemm: int, nmax_lu: int, nrhs_max: int, seed: int = 0,
                 device: str = "cuda:0"):
        import torch

        from . import inputs
        g = inputs.rng(seed)
        dev = torch.device(device)
        self.ga = torch.from_numpy(inputs.dd_uniform(nmax_gemm, nmax_gemm, g)).to(dev)
        self.gb = torch.from_numpy(inputs.dd_uniform(nmax_gemm, nmax_gemm, g)).to(dev)
        self.la = torch.from_numpy(inputs.dd_lu_matrix(nmax_lu, g)).to(dev)
        self.lb = torch.from_numpy(inputs.dd_uniform(nmax_lu, nrhs_max, g)).to(dev)
        self.nmax_gemm, self.nmax_lu = nmax_gemm, nmax_lu

    def payload(self, r: Request):
        rs = np.random.default_rng(r.rid)
        if r.kind == "gemm":
            o = int(rs.integers(0, self.nmax_gemm - r.n + 1))
            p = int(rs.integers(0, self.nmax_gemm - r.n + 1))
            return (self.ga[:, o:o + r.n, p:p + r.n], self.gb[:, p:p + r.n, o:o + r.n])
        o = int(rs.integers(0, self.nmax_lu - r.n + 1))
        return (self.la[:, o:o + r.n, o:o + r.n], self.lb[:, o:o + r.n, :r.nrhs])


def make_requests(trace) -> list:
    """Requests from inputs.serving_trace records (payloads attached later)."""
    return [Request(rid=k, kind=t["kind"], n=t["n"], nrhs=t["nrhs"], t_arrive=t["t_arrive"])
            for k, t in enumerate(trace)]
