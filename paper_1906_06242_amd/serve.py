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
waiting in a queue.  Results do not depend on the chunk a query starts at:
counts are exact in any order, and float64 sums of float32 weights are exact
in any order while partial sums stay below 2^53 of the smallest weight's ulp.

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
    """One submitted query and what happened to it."""
    qid: int
    query: object
    arrival: float
    admitted: float = math.nan
    done: float = math.nan
    slot: int = -1
    start_chunk: int = -1
    chunks_seen: int = 0
    hist_bytes: int = 0
    result: Optional[list] = None      # [(sumw, counts)] * 3 (host numpy)
    _snap: object = None

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def query_hist_bytes(q) -> int:
    """Device histogram memory of one query: float64 + uint64 per slot."""
    return 16 * q.n_scale * sum(len(e) + 1 for e in q.edges())


class GpuBackend:
    """Device side of the server: one plan, shared histograms, query slots."""

    def __init__(self, dd, n_chunks: int, n_slots: int, max_bins: int = 200, tune=None, stream=None):
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
        self.stream = stream or torch.cuda.current_stream()
        placeholder = datagen.Query()
        self.plan = H.Plan(self.chunks, [placeholder] * n_slots, tune, shared_hist=True,
                           reserve_bins=max_bins)
        self.sumw, self.counts = self.plan.new_hists()
        self.max_bins = max_bins
        for s in range(n_slots):
            self.plan.set_query(s, None, self.stream)
        self.blocks = []      # per slot: [(offset, nbins_capacity)] * 3
        for s in range(n_slots):
            self.blocks.append([self.plan.hist_offset(0, s, 0, h)[0] for h in range(3)])
        # pinned host staging for results, one per slot
        width = max_bins + 2
        self.pin_s = torch.zeros((n_slots, 3, width), dtype=torch.float64).pin_memory()
        self.pin_c = torch.zeros((n_slots, 3, width), dtype=torch.int64).pin_memory()
        self.launch_events: Deque = collections.deque()

    def set_query(self, slot: int, q) -> None:
        self.plan.set_query(slot, q, self.stream)

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

    def snapshot_and_clear(self, slot: int, q):
        """Enqueue: copy the slot's histograms to pinned host memory, then zero them."""
        torch = self.torch
        with torch.cuda.stream(self.stream):
            for h, e in enumerate(q.edges()):
                off, nb = self.blocks[slot][h], len(e) + 1
                self.pin_s[slot, h, :nb].copy_(self.sumw[off:off + nb], non_blocking=True)
                self.pin_c[slot, h, :nb].copy_(self.counts[off:off + nb], non_blocking=True)
                self.sumw[off:off + nb].zero_()
                self.counts[off:off + nb].zero_()
            ev = torch.cuda.Event()
            ev.record(self.stream)
        return ev

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
    """Continuous-batching scheduler over a backend with C chunks and S slots.

    hist_budget: device bytes of histograms that admitted queries may hold
    (admission stops when the next query would exceed it).
    max_ahead: launches allowed in flight before the host waits.
    """

    def __init__(self, backend, hist_budget: int = 1 << 30, max_ahead: int = 2,
                 clock: Callable[[], float] = time.perf_counter,
                 sleep: Callable[[float], None] = time.sleep):
        self.b = backend
        self.C = backend.n_chunks
        self.hist_budget = hist_budget
        self.max_ahead = max_ahead
        self.clock = clock
        self.sleep = sleep
        self.pending: Deque[Ticket] = collections.deque()
        self.free: List[int] = list(range(backend.n_slots))[::-1]
        self.active: Dict[int, Ticket] = {}
        self.finishing: List[Ticket] = []
        self.done: List[Ticket] = []
        self.chunk = 0
        self.hist_used = 0
        self.launches = 0
        self._qid = 0

    # -------------------------------------------------------------- interface
    def submit(self, q, arrival: Optional[float] = None) -> Ticket:
        t = Ticket(self._qid, q, self.clock() if arrival is None else arrival)
        t.hist_bytes = query_hist_bytes(q)
        self._qid += 1
        self.pending.append(t)
        return t

    def busy(self) -> bool:
        return bool(self.pending or self.active or self.finishing)

    def step(self) -> None:
        """Retire finished queries, admit waiting ones, launch one chunk pass."""
        self._collect()
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
            if self.active and self.hist_used + t.hist_bytes > self.hist_budget:
                break
            self.pending.popleft()
            t.slot = self.free.pop()
            t.admitted = self.clock()
            t.start_chunk = self.chunk
            self.hist_used += t.hist_bytes
            self.b.set_query(t.slot, t.query)
            self.active[t.slot] = t

    def _retire(self, t: Ticket) -> None:
        # a slot's host staging holds one result: collect an earlier one first
        for u in [u for u in self.finishing if u.slot == t.slot]:
            u.result = self.b.result(u.slot, u.query, u._snap)
            u.done = self.clock()
            self.done.append(u)
            self.finishing.remove(u)
        # stream order: this query's last pass, then the copy-out and clearing,
        # then the slot's next query
        t._snap = self.b.snapshot_and_clear(t.slot, t.query)
        self.b.set_query(t.slot, None)
        del self.active[t.slot]
        self.finishing.append(t)
        self.free.append(t.slot)
        self.hist_used -= t.hist_bytes

    def _collect(self) -> None:
        keep = []
        for t in self.finishing:
            if self.b.ready(t._snap):
                t.result = self.b.result(t.slot, t.query, t._snap)
                t.done = self.clock()
                self.done.append(t)
            else:
                keep.append(t)
        self.finishing = keep

    def _drain(self) -> None:
        while self.finishing:
            t = self.finishing.pop(0)
            t.result = self.b.result(t.slot, t.query, t._snap)
            t.done = self.clock()
            self.done.append(t)


def percentile(xs, p: float) -> float:
    xs = sorted(xs)
    if not xs:
        return math.nan
    k = (len(xs) - 1) * p / 100.0
    lo, hi = math.floor(k), math.ceil(k)
    return xs[lo] + (xs[hi] - xs[lo]) * (k - lo)
