"""Serving analysis queries over HBM-resident event columns, continuous batching.

The paper's motivation (Sec. I, Sec. IV) is fast iteration: many analysis
passes with different cuts and binnings over the same large dataset.  Here
the events stay resident on the GPU, split into C equal chunks; one launch of
the fused kernel makes a pass over one chunk for every query currently on the
device, so the chunks are scanned in a circle.  A query is admitted between
launches when a query slot and histogram memory are free, joins the scan at
the current chunk, and completes after C launches (every chunk seen once);
its histograms are then copied to the host and its slot is cleared and freed.
Queries arriving while others run therefore overlap on the device instead of
waiting in a queue.  Histogram memory is an arena of the device budget: each
admitted query's histograms are placed in a free range of it (first fit), so
the budget, not a fixed per-slot reservation, decides how many queries and
how many bins fit at once; a query larger than the whole arena is rejected.
A query can be cancelled, or given a deadline after which it is dropped
(waiting or running); its slot and arena range are then freed.

Results do not depend on the chunk a query starts at: counts are exact in any
order, and float64 sums of float32 weights are exact in any order while
partial sums stay below 2^53 of the smallest weight's ulp.

Scheduler and device are separated by a small backend interface
(GpuBackend here), so the scheduling logic can be exercised without a GPU.
"""
from __future__ import annotations

import collections
import math
import time
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional


@dataclass
class Ticket:
    """One submitted query and what happened to it.

    status: pending, active, finishing, done, cancelled, timeout, rejected.
    Times: arrival, admitted (a slot and an arena range given), retired (its
    last chunk pass enqueued), done (histograms on the host, or dropped)."""
    qid: int
    query: object
    arrival: float
    deadline: float = math.inf
    status: str = "pending"
    admitted: float = math.nan
    retired: float = math.nan
    done: float = math.nan
    slot: int = -1
    at: int = -1                       # first histogram slot in the arena
    start_chunk: int = -1
    chunks_seen: int = 0
    hist_bytes: int = 0
    result: Optional[list] = None      # [(sumw, counts)] * 3 (host numpy)
    _snap: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival

    @property
    def queue_wait(self) -> float:
        return self.admitted - self.arrival

    @property
    def scan(self) -> float:
        return self.retired - self.admitted

    @property
    def copy_out(self) -> float:
        return self.done - self.retired


def query_slots(q) -> int:
    """Histogram slots of one query: nbins + 2 per observable and scale."""
    return q.n_scale * sum(len(e) + 1 for e in q.edges())


def query_hist_bytes(q) -> int:
    """Device histogram memory of one query: float64 + uint64 per slot."""
    return 16 * query_slots(q)


class Arena:
    """First-fit allocator of histogram slots [0, size) with coalescing."""

    def __init__(self, size: int):
        self.size = size
        self.free = [(0, size)] if size > 0 else []   # sorted (start, length)

    def alloc(self, n: int) -> int:
        for i, (a, m) in enumerate(self.free):
            if m >= n:
                if m == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (a + n, m - n)
                return a
        return -1

    def release(self, a: int, n: int) -> None:
        self.free.append((a, n))
        self.free.sort()
        merged = []
        for s, m in self.free:
            if merged and merged[-1][0] + merged[-1][1] == s:
                merged[-1] = (merged[-1][0], merged[-1][1] + m)
            else:
                merged.append((s, m))
        self.free = merged

    def used(self) -> int:
        return self.size - sum(m for _, m in self.free)


class GpuBackend:
    """Device side of the server: one plan over the chunks, query slots, and
    one histogram arena of hist_budget bytes shared by the admitted queries
    (each placed by the scheduler); queries may have up to max_bins bins per
    histogram."""

    def __init__(self, dd, n_chunks: int, n_slots: int, hist_budget: int = 1 << 26, max_bins: int = 2000,
                 tune=None, stream=None):
        import torch
        from . import datagen
        from . import hepk as H
        self.H = H
        self.torch = torch
        n = dd.n_events
        bounds = [n * c // n_chunks for c in range(n_chunks + 1)]
        self.chunks = [dd.view(bounds[c], bounds[c + 1]) for c in range(n_chunks)]
        self.n_chunks = n_chunks
        self.n_slots = n_slots
        self.arena_slots = hist_budget // 16
        self.stream = stream or torch.cuda.current_stream()
        placeholder = datagen.Query()
        self.plan = H.Plan(self.chunks, [placeholder] * n_slots, tune, shared_hist=True,
                           reserve_bins=max_bins, hist_arena_slots=self.arena_slots)
        self.sumw, self.counts = self.plan.new_hists()
        self.max_bins = max_bins
        for s in range(n_slots):
            self.plan.set_query(s, None, self.stream)
        # pinned host staging for results, one per slot
        width = max_bins + 2
        self.pin_s = torch.zeros((n_slots, 3, width), dtype=torch.float64).pin_memory()
        self.pin_c = torch.zeros((n_slots, 3, width), dtype=torch.int64).pin_memory()
        self.launch_events: Deque = collections.deque()

    def set_query(self, slot: int, q, at: int = -1) -> None:
        self.plan.set_query(slot, q, self.stream, at=None if q is None or at < 0 else at)

    def launch(self, chunk: int) -> None:
        torch = self.torch
        with torch.cuda.stream(self.stream):
            self.plan.run_range(chunk, 1, self.sumw, self.counts, self.stream)
            ev = torch.cuda.Event()
            ev.record(self.stream)
        self.launch_events.append(ev)

    def in_flight(self) -> int:
        while self.launch_events and self.launch_events[0].query():
            self.launch_events.popleft()
        return len(self.launch_events)

    def wait_one(self) -> None:
        if self.launch_events:
            self.launch_events.popleft().synchronize()

    def _blocks(self, q, at: int):
        off = at
        for e in q.edges():
            nb = len(e) + 1
            yield off, nb
            off += nb

    def snapshot_and_clear(self, slot: int, q, at: int):
        """Enqueue: copy the query's histograms to the slot's pinned host
        memory, then zero its arena range."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            for h, (off, nb) in enumerate(self._blocks(q, at)):
                self.pin_s[slot, h, :nb].copy_(self.sumw[off:off + nb], non_blocking=True)
                self.pin_c[slot, h, :nb].copy_(self.counts[off:off + nb], non_blocking=True)
            self.sumw[at:at + query_slots(q)].zero_()
            self.counts[at:at + query_slots(q)].zero_()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return ev

    def clear(self, slot: int, q, at: int) -> None:
        """Enqueue: zero a dropped query's arena range (after its passes)."""
        with self.torch.cuda.stream(self.stream):
            self.sumw[at:at + query_slots(q)].zero_()
            self.counts[at:at + query_slots(q)].zero_()

    def ready(self, snap) -> bool:
        return snap.query()

    def result(self, slot: int, q, snap) -> list:
        snap.synchronize()
        out = []
        for h, e in enumerate(q.edges()):
            nb = len(e) + 1
            out.append((self.pin_s[slot, h, :nb].numpy().copy(),
                        self.pin_c[slot, h, :nb].numpy().view("uint64").copy()))
        return out

    def close(self):
        self.torch.cuda.synchronize()
        self.plan.close()


class Server:
    """Continuous-batching scheduler over a backend with C chunks, S slots and
    a histogram arena of backend.arena_slots slots.

    hist_budget: device bytes of histograms that admitted queries may hold
    (at most the arena; admission stops when the next query's range does not
    fit).  timeout: seconds after arrival after which a query that has not
    finished is dropped (None: never).  max_ahead: launches allowed in flight
    before the host waits.
    """

    def __init__(self, backend, hist_budget: Optional[int] = None, max_ahead: int = 2,
                 timeout: Optional[float] = None,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.b = backend
        self.C = backend.n_chunks
        arena = backend.arena_slots if hist_budget is None else min(backend.arena_slots, hist_budget // 16)
        self.arena = Arena(arena)
        self.hist_budget = 16 * arena
        self.max_ahead = max_ahead
        self.timeout = timeout
        self.clock = clock
        self.sleep = sleep
        self.pending: Deque[Ticket] = collections.deque()
        self.free: List[int] = list(range(backend.n_slots))[::-1]
        self.active: Dict[int, Ticket] = {}
        self.finishing: List[Ticket] = []
        self.done: List[Ticket] = []
        self.dropped: List[Ticket] = []
        self.chunk = 0
        self.launches = 0
        self._qid = 0

    @property
    def hist_used(self) -> int:
        return 16 * self.arena.used()

    # -------------------------------------------------------------- interface
    def submit(self, q, arrival: Optional[float] = None, timeout: Optional[float] = None) -> Ticket:
        t = Ticket(self._qid, q, self.clock() if arrival is None else arrival)
        t.hist_bytes = query_hist_bytes(q)
        limit = self.timeout if timeout is None else timeout
        if limit is not None:
            t.deadline = t.arrival + limit
        self._qid += 1
        if query_slots(q) > self.arena.size:
            self._drop(t, "rejected")
        else:
            self.pending.append(t)
        return t

    def cancel(self, t: Ticket) -> bool:
        """Drops a waiting or running query (False if it already finished)."""
        if t.status == "pending":
            self.pending.remove(t)
            self._drop(t, "cancelled")
            return True
        if t.status == "active":
            self._stop(t, "cancelled")
            return True
        return False

    def busy(self) -> bool:
        return bool(self.pending or self.active or self.finishing)

    def step(self) -> None:
        """Retire finished queries, drop expired ones, admit waiting ones,
        launch one chunk pass."""
        self._collect()
        self._expire()
        self._admit()
        if self.active:
            while self.b.in_flight() >= self.max_ahead:
                self.b.wait_one()
                self._collect()
            self.b.launch(self.chunk)
            self.launches += 1
            for t in list(self.active.values()):
                t.chunks_seen += 1
                if t.chunks_seen == self.C:
                    self._retire(t)
            self.chunk = (self.chunk + 1) % self.C

    def run_stream(self, queries, t0: Optional[float] = None) -> List[Ticket]:
        """Open loop: query i arrives at t0 + queries[i].arrival; runs until all are done."""
        t0 = self.clock() if t0 is None else t0
        order = sorted(queries, key=lambda q: q.arrival)
        i = 0
        while i < len(order) or self.busy():
            now = self.clock()
            while i < len(order) and t0 + order[i].arrival <= now:
                self.submit(order[i], t0 + order[i].arrival)
                i += 1
            if self.busy():
                self.step()
            elif i < len(order):
                self.sleep(max(0.0, t0 + order[i].arrival - self.clock()))
        self._drain()
        return self.done

    def run_closed(self, queries) -> List[Ticket]:
        """Closed loop: every query is waiting at the start."""
        now = self.clock()
        for q in queries:
            self.submit(q, now)
        while self.busy():
            self.step()
        self._drain()
        return self.done

    # -------------------------------------------------------------- internals
    def _admit(self) -> None:
        while self.pending and self.free:
            t = self.pending[0]
            at = self.arena.alloc(query_slots(t.query))
            if at < 0:
                break  # its histograms do not fit until running queries finish
            self.pending.popleft()
            t.slot = self.free.pop()
            t.at = at
            t.status = "active"
            t.admitted = self.clock()
            t.start_chunk = self.chunk
            self.b.set_query(t.slot, t.query, at)
            self.active[t.slot] = t

    def _expire(self) -> None:
        now = self.clock()
        for t in [t for t in self.pending if t.deadline <= now]:
            self.pending.remove(t)
            self._drop(t, "timeout")
        for t in [t for t in self.active.values() if t.deadline <= now]:
            self._stop(t, "timeout")

    def _drop(self, t: Ticket, why: str) -> None:
        t.status = why
        t.done = self.clock()
        self.dropped.append(t)

    def _stop(self, t: Ticket, why: str) -> None:
        # stream order: the passes already enqueued, then the slot goes idle
        # and the range is zeroed, then it may be given to another query
        self.b.set_query(t.slot, None)
        self.b.clear(t.slot, t.query, t.at)
        del self.active[t.slot]
        self.free.append(t.slot)
        self.arena.release(t.at, query_slots(t.query))
        self._drop(t, why)

    def _retire(self, t: Ticket) -> None:
        # a slot's host staging holds one result: collect an earlier one first
        for u in [u for u in self.finishing if u.slot == t.slot]:
            self._finish(u, self.b.result(u.slot, u.query, u._snap))
            self.finishing.remove(u)
        # stream order: this query's last pass, then the copy-out and clearing,
        # then the slot's next query
        t.retired = self.clock()
        t._snap = self.b.snapshot_and_clear(t.slot, t.query, t.at)
        self.b.set_query(t.slot, None)
        del self.active[t.slot]
        t.status = "finishing"
        self.finishing.append(t)
        self.free.append(t.slot)
        self.arena.release(t.at, query_slots(t.query))

    def _finish(self, t: Ticket, result) -> None:
        t.result = result
        t.done = self.clock()
        t.status = "done"
        self.done.append(t)

    def _collect(self) -> None:
        keep = []
        for t in self.finishing:
            if self.b.ready(t._snap):
                self._finish(t, self.b.result(t.slot, t.query, t._snap))
            else:
                keep.append(t)
        self.finishing = keep

    def _drain(self) -> None:
        while self.finishing:
            t = self.finishing.pop(0)
            self._finish(t, self.b.result(t.slot, t.query, t._snap))


def percentile(xs, p: float) -> float:
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
