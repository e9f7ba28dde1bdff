"""Continuous-batching server for GBS probability requests.

Requests (output patterns, i.e. mode lists) arrive at any time. The server keeps the GBS state
(U, B) resident on the device and runs a loop of *steps*. Each step is one launch of
``gbs_prob_slices`` over a mix of work from every admitted request:

* Every pattern's 2^(n/2) - 1 subset terms are cut into slices whose boundaries depend only on n,
  so a long request (n = 32: 65,535 subsets) is spread over several steps while short ones
  (n = 8: 15 subsets) finish in one, and a request's result is the same whatever it was batched
  with (each slice partial depends only on its pattern and range; slices are combined in order).
* Admission is by device memory: a request needs one 32-byte partial per slice in a fixed device
  pool; requests wait when the pool or the active-request table is full and are admitted as
  earlier ones complete. A request that could never fit is rejected.
* A step takes slices from active requests, shortest remaining work first, at most ``step_flops``
  of modelled work and at most ``share`` of that from one request, so short requests are not held
  behind long ones; the oldest active request always gets one slice outside the budget and then
  competes for the rest like the others, so long ones keep moving. Up to ``inflight`` steps are
  queued on the stream, so the host prepares the next step while the device runs the current one.
* When a request's last slice has been launched, a ``gbs_finalize`` launch (its slices' partials,
  in slice order, compensated) follows on the same stream and produces the probability; the
  request completes when that result has been copied back.

``FifoServer`` is the comparison path: one request at a time through the plain per-pattern GPU
path (``gbs_prob_batch`` with eager, non-persistent launches), in arrival order.
"""
from __future__ import annotations

import collections
import dataclasses
import gc
import threading
import time
from concurrent.futures import Future
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np

PARTIAL_BYTES = 32  # one gbs_partial


def slice_plan(n: int, max_slice: int = 4096) -> List[tuple]:
    """Slice boundaries [lo, hi) of a size-n pattern's subset order (a function of n only)."""
    if n <= 0 or n % 2:
        return []
    cnt = (1 << (n // 2)) - 1
    return [(lo, min(cnt, lo + max_slice)) for lo in range(0, cnt, max_slice)]


def subset_flops(n: int, lo: int, hi: int, haf_flops: Callable[[int], float]) -> float:
    """Modelled work of a slice: its share of the pattern's flops (by subset count)."""
    cnt = (1 << (n // 2)) - 1
    return haf_flops(n) * (hi - lo) / max(cnt, 1)


@dataclasses.dataclass(eq=False)  # requests are distinct objects: identity equality (cheap list removal)
class Request:
    rid: int
    modes: np.ndarray
    n: int
    t_arrival: float
    future: Future
    slices: List[tuple] = dataclasses.field(default_factory=list)
    work: List[float] = dataclasses.field(default_factory=list)  # modelled flops of each slice
    remaining: float = 0.0      # modelled flops of the slices not yet issued
    next_slice: int = 0
    pool_off: int = -1          # first partial slot in the device pool
    t_done: float = 0.0


def hold_gc():
    """Collect once, freeze what is alive and switch automatic collection off."""
    gc.collect()
    gc.freeze()
    gc.disable()


def release_gc():
    gc.enable()
    gc.unfreeze()


class SliceBackend:
    """What the server needs from the device. GpuBackend is the real one; tests use fakes.

    launch_step(jobs, finished) enqueues the slices of one step -- jobs are
    (modes, lo, hi, pool_index) -- followed by the finalize of the requests whose last slice is in
    this (or an earlier) step, and returns a handle; done(handle) polls it; results(handle) gives the
    finished requests' probabilities in order.
    """

    def launch_step(self, jobs: List[tuple], finished: List[Request]) -> object:
        raise NotImplementedError

    def done(self, handle) -> bool:
        raise NotImplementedError

    def results(self, handle) -> np.ndarray:
        raise NotImplementedError

    def haf_flops(self, n: int) -> float:
        return float(2 ** (n // 2)) * max(n, 2) ** 3


class GpuBackend(SliceBackend):
    """libgbs on one device: slices into a device partial pool, one finalize launch per step.

    Within a step, the kernels of the different (engine, subset size) variants run side by side on
    `streams_per_call` streams (gbs_ctx_set_streams): a step holds many sizes with a few patterns each,
    and one small kernel at a time leaves most of the device idle (measured at 0.8 of capacity:
    median latency 79 ms on one stream, 18 ms on four). Consecutive steps go round-robin to `lanes`
    (context, stream) pairs, so one step's kernels can start while the previous step's last kernels
    drain (no gain measured at two lanes; one is the default). Each context has its own workspace;
    the partial pool and the state are shared (requests own disjoint pool slots). A step's finalize
    waits for the previous step's slices (on the other stream): a request's slices are all in that
    step or earlier ones, and earlier steps on either stream complete before it in stream order."""

    def __init__(self, ctx, state, pool_entries: int, max_finish: int = 4096, ring: int = 8, stream=None,
                 lanes: int = 1, streams_per_call: int = 4):
        import torch
        from . import gbs
        self._gbs = gbs
        self.ctx = ctx
        self.state = state
        self.torch = torch
        streams = [stream or torch.cuda.Stream(device=ctx.torch_device)]
        ctxs = [ctx]
        for _ in range(1, max(1, lanes)):
            streams.append(torch.cuda.Stream(device=ctx.torch_device))
            ctxs.append(gbs.Context(ctx.device, use_graph=False))
            ctxs[-1]._copy_tuning_from(ctx)
            ctxs[-1].set_precision(ctx.precision)
        for c in ctxs:  # a step's kernels for the different (engine, k) variants run side by side
            c.set_streams(streams_per_call)
        self.lanes = list(zip(ctxs, streams))
        self._lane = 0
        self._prev_slices = None  # event after the previous step's slices
        self.pool = torch.zeros((pool_entries, 4), dtype=torch.float64, device=ctx.torch_device)
        self.ring = ring
        self.max_finish = max_finish
        self.prob = torch.zeros((ring, max_finish), dtype=torch.float64, device=ctx.torch_device)
        self.host = torch.zeros((ring, max_finish), dtype=torch.float64).pin_memory()
        self._slot = 0

    @property
    def stream(self):
        return self.lanes[0][1]

    def warmup(self, sizes):
        """One pattern of every size in `sizes` through each lane, so the first real steps do not pay
        for loading kernels and allocating staging memory."""
        for ctx, stream in self.lanes:
            for n in sizes:
                ctx.prob_batch(self.state, [list(range(n))], stream=stream)
        self.torch.cuda.synchronize()

    def haf_flops(self, n: int) -> float:
        return self._gbs.haf_flops(n) if n > 0 and n % 2 == 0 else 0.0

    @staticmethod
    def _pack(mode_lists):
        lens = np.fromiter((len(m) for m in mode_lists), dtype=np.int64, count=len(mode_lists))
        offsets = np.zeros(len(mode_lists) + 1, dtype=np.int64)
        np.cumsum(lens, out=offsets[1:])
        modes = np.concatenate(mode_lists) if len(mode_lists) else np.zeros(0, np.int32)
        return np.ascontiguousarray(modes, dtype=np.int32), offsets

    def launch_step(self, jobs, finished):
        torch = self.torch
        ctx, stream = self.lanes[self._lane]
        self._lane = (self._lane + 1) % len(self.lanes)
        if jobs:
            packed = self._pack([j[0] for j in jobs])
            rng = np.array([(j[1], j[2], j[3]) for j in jobs], dtype=np.int64).reshape(-1, 3)
            ctx.prob_slices(self.state, packed, rng[:, 0], rng[:, 1], partials_out=self.pool, out_idx=rng[:, 2],
                            stream=stream)
        prev = self._prev_slices
        ev_slices = torch.cuda.Event()
        ev_slices.record(stream)
        self._prev_slices = ev_slices
        slot = self._slot
        self._slot = (self._slot + 1) % self.ring
        nf = len(finished)
        if nf > self.max_finish:
            raise ValueError("too many requests finishing in one step")
        if nf:
            if prev is not None:
                stream.wait_event(prev)
            lo = [r.pool_off for r in finished]
            hi = [r.pool_off + len(r.slices) for r in finished]
            ctx.finalize(self.state, self.pool, lo, hi, self._pack([r.modes for r in finished]), want_prob=True,
                         prob_out=self.prob[slot, :nf], want_haf=False, stream=stream)
            with torch.cuda.stream(stream):
                self.host[slot, :nf].copy_(self.prob[slot, :nf], non_blocking=True)
        ev = torch.cuda.Event()
        ev.record(stream)
        return (ev, slot, nf)

    def done(self, handle) -> bool:
        return handle[0].query()

    def results(self, handle) -> np.ndarray:
        _, slot, nf = handle
        return self.host[slot, :nf].numpy().copy()


class Server:
    """Continuous batching over a SliceBackend. Thread-safe submit(); run in a background thread."""

    def __init__(self, backend: SliceBackend, pool_entries: int, max_active: int = 8192,
                 step_flops: float = 1e11, share: float = 0.5, inflight: int = 3, max_slice: int = 4096,
                 max_finish: int = 4096, hold_gc: bool = False, adaptive: bool = True):
        """hold_gc: while the server runs, freeze the objects alive at start() and switch off Python's
        cyclic garbage collector (switched back on at stop()). Its full collections pause every
        thread for tens of milliseconds once tens of thousands of requests and futures are alive,
        and the device idles meanwhile; a serving process that does not create reference cycles
        loses nothing by deferring them."""
        self.b = backend
        self.hold_gc = hold_gc
        self._gc_was_enabled = None
        self.pool_entries = pool_entries
        self.max_active = max_active
        self.step_flops = step_flops
        # adaptive: a step takes at least its share of the backlog (the active requests' remaining work
        # over the steps in flight), so steps grow with the load and the device's efficiency with them
        self.adaptive = adaptive
        self.share = share
        self.inflight = inflight
        self.max_slice = max_slice
        self.max_finish = max_finish
        self._lock = threading.Lock()
        self._pending: collections.deque = collections.deque()
        self._active: List[Request] = []
        self._steps: collections.deque = collections.deque()  # (handle, finished requests)
        self._free_pool = [(0, pool_entries)]  # free ranges (offset, length)
        self._rid = 0
        self._flops_cache: Dict[int, float] = {}
        self._stop = False
        self._thread: Optional[threading.Thread] = None
        self.latencies: List[float] = []
        self.records: List[tuple] = []  # (rid, t_arrival, t_done) of completed requests
        self.completed = 0
        self.rejected = 0
        self.failed = 0
        self.steps = 0
        self.max_concurrent = 0
        self.arrivals_in_flight = 0  # requests submitted while a step was on the device
        self.memory_waits = 0        # admission attempts that found the pool too full
        self.host_build_s = 0.0      # host time building steps (scheduling)
        self.host_launch_s = 0.0     # host time enqueueing steps (marshalling, planning, staging)
        self._t_first = None
        self._t_last = None

    # ------------------------------------------------------------ public API
    def submit(self, modes: Sequence[int], t_arrival: Optional[float] = None) -> Future:
        """Queue a request; t_arrival (time.perf_counter() seconds) is when it arrived, default now:
        latency is measured from it."""
        f: Future = Future()
        m = np.ascontiguousarray(modes, dtype=np.int32)
        t = time.perf_counter() if t_arrival is None else t_arrival
        with self._lock:
            r = Request(self._rid, m, len(m), t, f)
            self._rid += 1
            r.slices = slice_plan(r.n, self.max_slice)
            r.work = [subset_flops(r.n, lo, hi, self._haf_flops) for lo, hi in r.slices]
            r.remaining = sum(r.work)
            if len(r.slices) > self.pool_entries:
                self.rejected += 1
                f.set_exception(MemoryError(f"request needs {len(r.slices)} partial slots, pool has {self.pool_entries}"))
                return f
            self._pending.append(r)
            if self._steps:
                self.arrivals_in_flight += 1
            if self._t_first is None:
                self._t_first = r.t_arrival
        return f

    def start(self):
        if self.hold_gc:
            hold_gc()
        self._thread = threading.Thread(target=self._loop, name="gbs-server", daemon=True)
        self._thread.start()
        return self

    def idle(self) -> bool:
        with self._lock:
            return not (self._pending or self._active or self._steps)

    def stop(self, drain: bool = True, timeout: float = 60.0):
        if drain:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < timeout and not self.idle():
                time.sleep(0.001)
        self._stop = True
        if self._thread:
            self._thread.join(timeout)
        if self.hold_gc:
            release_gc()

    def latencies_by_rid(self, skip: int = 0) -> List[float]:
        """Latencies (s) of the completed requests numbered skip and later (the first `skip` are warm-up)."""
        return [t1 - t0 for rid, t0, t1 in self.records if rid >= skip]

    def completion_rate(self, skip: int = 0) -> float:
        """Completed requests per second among those numbered skip and later: (count - 1) over the time
        from their first completion to their last (equals the arrival rate while the server keeps up)."""
        done = sorted(t1 for rid, t0, t1 in self.records if rid >= skip)
        return (len(done) - 1) / (done[-1] - done[0]) if len(done) > 1 and done[-1] > done[0] else float("nan")

    def span(self, skip: int = 0) -> float:
        """Seconds from the arrival of the first request numbered >= skip to the last completion."""
        recs = [r for r in self.records if r[0] >= skip]
        return max(r[2] for r in recs) - min(r[1] for r in recs) if recs else float("nan")

    def stats(self) -> Dict[str, float]:
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        span = (self._t_last - self._t_first) if (self._t_last and self._t_first) else float("nan")
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "completed": self.completed, "rejected": self.rejected,
                "failed": self.failed, "throughput_req_s": self.completed / span if span == span and span > 0 else 0.0,
                "steps": self.steps, "max_concurrent": self.max_concurrent,
                "arrivals_in_flight": self.arrivals_in_flight, "memory_waits": self.memory_waits,
                "host_build_ms_per_step": 1e3 * self.host_build_s / max(self.steps, 1),
                "host_launch_ms_per_step": 1e3 * self.host_launch_s / max(self.steps, 1)}

    # ------------------------------------------------------------ internals
    def _alloc_pool(self, need: int) -> int:
        for i, (off, ln) in enumerate(self._free_pool):
            if ln >= need:
                if ln == need:
                    self._free_pool.pop(i)
                else:
                    self._free_pool[i] = (off + need, ln - need)
                return off
        return -1

    def _free_pool_range(self, off: int, ln: int):
        if ln <= 0:
            return
        self._free_pool.append((off, ln))
        self._free_pool.sort()
        merged = []
        for o, l in self._free_pool:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + l)
            else:
                merged.append((o, l))
        self._free_pool = merged

    def _admit(self):
        while self._pending and len(self._active) < self.max_active:
            r = self._pending[0]
            need = len(r.slices)
            off = self._alloc_pool(need) if need else 0
            if off < 0:
                self.memory_waits += 1
                break  # wait for device memory to free up
            self._pending.popleft()
            r.pool_off = off
            self._active.append(r)
        self.max_concurrent = max(self.max_concurrent, len(self._active))

    def _haf_flops(self, n: int) -> float:
        """The backend's flop model for size n, asked once per n."""
        v = self._flops_cache.get(n)
        if v is None:
            v = self._flops_cache[n] = float(self.b.haf_flops(n))
        return v

    def _build_step(self):
        """Shortest remaining work first (short requests are not held behind long ones), each request at
        most `share` of the step budget, and the oldest active request always gets a slice so long
        requests keep moving under load."""
        jobs, finished = [], []
        budget = self.step_flops
        if self.adaptive:
            budget = max(budget, sum(r.remaining for r in self._active) / self.inflight)
        cap = budget * self.share
        order = sorted(self._active, key=lambda r: (r.remaining, r.rid))
        oldest = min(self._active, key=lambda r: r.rid)
        if order and order[0] is not oldest:
            order.remove(oldest)
            order.insert(0, oldest)
        for r in order:
            if len(finished) >= self.max_finish:
                break
            # the oldest request gets one slice even when the budget is spent, then draws from the
            # budget like the others
            first_free = r is oldest and len(order) > 1
            if budget <= 0 and not first_free:
                continue
            used = 0.0
            while r.next_slice < len(r.slices) and (first_free or (budget > 0 and (used < cap or used == 0.0))):
                lo, hi = r.slices[r.next_slice]
                w = r.work[r.next_slice]
                jobs.append((r.modes, lo, hi, r.pool_off + r.next_slice))
                r.next_slice += 1
                r.remaining -= w
                used += w  # the request's own share counts every slice
                if first_free:
                    first_free = False
                    continue  # outside the step budget
                budget -= w
            if r.next_slice == len(r.slices):
                finished.append(r)
        if finished:
            done = {id(r) for r in finished}
            self._active = [r for r in self._active if id(r) not in done]
        return jobs, finished

    def _complete(self, reqs: List[Request], probs: Optional[np.ndarray], err: Optional[BaseException]):
        now = time.perf_counter()
        for i, r in enumerate(reqs):
            self._free_pool_range(r.pool_off, len(r.slices))
            if err is not None:
                self.failed += 1
                r.future.set_exception(err)
            else:
                r.t_done = now
                self.latencies.append(now - r.t_arrival)
                self.records.append((r.rid, r.t_arrival, now))
                self.completed += 1
                r.future.set_result(float(probs[i]))
            self._t_last = now

    def _loop(self):
        while not self._stop:
            progressed = False
            with self._lock:
                while self._steps and self.b.done(self._steps[0][0]):
                    h, reqs = self._steps.popleft()
                    if reqs:
                        self._complete(reqs, self.b.results(h), None)
                    progressed = True
                self._admit()
                jobs, finished = ([], [])
                if len(self._steps) < self.inflight and self._active:
                    tb = time.perf_counter()
                    jobs, finished = self._build_step()
                    self.host_build_s += time.perf_counter() - tb
            if jobs or finished:
                try:
                    tl = time.perf_counter()
                    h = self.b.launch_step(jobs, finished)
                    self.host_launch_s += time.perf_counter() - tl
                    with self._lock:
                        self.steps += 1
                        self._steps.append((h, finished))
                except Exception as e:  # a failed launch fails the requests it carried, serving goes on
                    with self._lock:
                        self._complete(finished, None, e)
                        hit = {id(j[0]) for j in jobs}
                        for r in list(self._active):
                            if id(r.modes) in hit:
                                self._active.remove(r)
                                self._complete([r], None, e)
                progressed = True
            if not progressed:
                time.sleep(0.0001)


class FifoServer:
    """One request at a time through the per-pattern GPU path (the comparison for serving)."""

    def __init__(self, ctx, state):
        self.ctx = ctx
        self.state = state
        self._q: collections.deque = collections.deque()
        self._lock = threading.Lock()
        self._stop = False
        self.latencies: List[float] = []
        self.records: List[tuple] = []  # (rid, t_arrival, t_done)
        self.completed = 0
        self._rid = 0
        self._t_first = None
        self._t_last = None

    def submit(self, modes, t_arrival: Optional[float] = None) -> Future:
        f: Future = Future()
        with self._lock:
            t = time.perf_counter() if t_arrival is None else t_arrival
            self._q.append((np.asarray(modes, dtype=np.int32), t, f, self._rid))
            self._rid += 1
            if self._t_first is None:
                self._t_first = t
        return f

    latencies_by_rid = Server.latencies_by_rid
    completion_rate = Server.completion_rate
    span = Server.span

    def start(self):
        self._thread = threading.Thread(target=self._loop, daemon=True)
        self._thread.start()
        return self

    def stop(self, drain=True, timeout=120.0):
        if drain:
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < timeout:
                with self._lock:
                    if not self._q:
                        break
                time.sleep(0.001)
        self._stop = True
        self._thread.join(timeout)

    def _loop(self):
        import torch
        while not self._stop:
            with self._lock:
                item = self._q.popleft() if self._q else None
            if item is None:
                time.sleep(0.0001)
                continue
            modes, t0, f, rid = item
            try:
                p = self.ctx.prob_batch(self.state, [modes])
                v = float(p.cpu().item())
                now = time.perf_counter()
                self.latencies.append(now - t0)
                self.records.append((rid, t0, now))
                self.completed += 1
                self._t_last = now
                f.set_result(v)
            except Exception as e:
                f.set_exception(e)

    def stats(self):
        lat = np.array(self.latencies) if self.latencies else np.zeros(1)
        span = (self._t_last - self._t_first) if (self._t_last and self._t_first) else float("nan")
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "mean_ms": float(lat.mean() * 1e3), "completed": self.completed,
                "throughput_req_s": self.completed / span if span == span and span > 0 else 0.0}


def replay(server, arrivals: np.ndarray, patterns: Sequence[Sequence[int]], warmup: int = 0):
    """Submit patterns at the given arrival times (seconds from start) in real time; returns futures.

    Every request whose arrival time has passed is submitted at once with that arrival time, then the
    feeder sleeps until the next one (sleeping releases the interpreter lock, so the feeder does not
    compete with the server thread); latencies count from the scheduled arrival."""
    futs = []
    t0 = time.perf_counter()
    i, total = 0, len(arrivals)
    while i < total:
        now = time.perf_counter() - t0
        while i < total and arrivals[i] <= now:
            futs.append(server.submit(patterns[i], t_arrival=t0 + float(arrivals[i])))
            i += 1
        if i < total:
            time.sleep(max(0.0, float(arrivals[i]) - (time.perf_counter() - t0)))
    return futs
