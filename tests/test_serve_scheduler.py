"""The serving scheduler on the CPU: the oracle as the device, a fake clock.

Checks continuous batching: queries are admitted as slots and histogram
memory free up, every query sees every chunk exactly once whatever chunk it
starts at, results equal the oracle's full pass for that query alone, and
latency bookkeeping follows the clock.
"""
import numpy as np

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd.serve import Arena, Server, percentile, query_hist_bytes, query_slots


def host_slice(ds, e0, e1):
    def cut(c):
        a, b = int(c.offsets[e0]), int(c.offsets[e1])
        return datagen.Collection(c.offsets[e0:e1 + 1] - a, {k: v[a:b] for k, v in c.cols.items()})
    return datagen.Dataset(e1 - e0, cut(ds.jets), cut(ds.muons), ds.weight[e0:e1],
                           cut(ds.electrons) if ds.electrons is not None else None, ds.content_dtype)


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 0.0)


class OracleBackend:
    """Synchronous stand-in for the GPU: each launch runs the oracle on one chunk."""

    def __init__(self, ds, n_chunks, n_slots, clock, launch_time=0.001, arena_slots=1 << 22):
        self.arena_slots = arena_slots
        self.ranges = {}  # slot -> (at, n) of the installed query
        self.arena_peak = []  # arena slots in use at each launch
        n = ds.n_events
        b = [n * c // n_chunks for c in range(n_chunks + 1)]
        self.chunks = [host_slice(ds, b[c], b[c + 1]) for c in range(n_chunks)]
        self.n_chunks, self.n_slots = n_chunks, n_slots
        self.q = [None] * n_slots
        self.h = [None] * n_slots
        self.clock, self.launch_time = clock, launch_time
        self.log = []

    def set_query(self, slot, q, at=-1):
        self.q[slot] = q
        if q is not None:
            self.h[slot] = [(np.zeros(len(e) + 1), np.zeros(len(e) + 1, np.uint64)) for e in q.edges()]
            # the scheduler's placements never overlap, and stay in the arena
            n = query_slots(q)
            assert 0 <= at and at + n <= self.arena_slots
            for s2, (a2, n2) in self.ranges.items():
                assert s2 == slot or at + n <= a2 or a2 + n2 <= at, "overlapping arena ranges"
            self.ranges[slot] = (at, n)
        else:
            self.ranges.pop(slot, None)
        self.log.append(("set", slot, q is not None))

    def launch(self, c):
        self.arena_peak.append(sum(n for _, n in self.ranges.values()))
        self.clock.t += self.launch_time
        active = [s for s in range(self.n_slots) if self.q[s] is not None]
        self.log.append(("launch", c, tuple(active)))
        for s in active:
            got = ref.pipeline(self.chunks[c], [self.q[s]])[0][0]
            self.h[s] = [(a[0] + g[0], a[1] + g[1]) for a, g in zip(self.h[s], got)]

    def in_flight(self):
        return 0

    def wait_one(self):
        pass

    def clear(self, slot, q, at):
        self.log.append(("clear", slot, at))

    def snapshot_and_clear(self, slot, q, at):
        snap = [(s.copy(), c.copy()) for s, c in self.h[slot]]
        self.h[slot] = [(np.zeros_like(s), np.zeros_like(c)) for s, c in self.h[slot]]
        return snap

    def ready(self, snap):
        return True

    def result(self, slot, q, snap):
        return snap


def run_server(n_slots=3, budget=1 << 30, qps=300.0, n_q=10, C=5):
    ds = datagen.make_dataset(7, 6000)
    clock = FakeClock()
    be = OracleBackend(ds, C, n_slots, clock, arena_slots=budget // 16)
    srv = Server(be, clock=clock, sleep=clock.sleep)
    qs = datagen.draw_queries(11, n_q, qps=qps)
    done = srv.run_stream(qs, t0=0.0)
    return ds, qs, done, be, srv


def test_every_query_matches_its_alone_oracle_pass():
    ds, qs, done, be, srv = run_server()
    assert len(done) == len(qs)
    for t in done:
        want = ref.pipeline(ds, [t.query])[0][0]
        for h in range(3):
            assert np.array_equal(t.result[h][1], want[h][1])
            assert np.array_equal(t.result[h][0], want[h][0])
        assert t.chunks_seen == be.n_chunks
    # queries joined the circular scan at different chunks
    assert len({t.start_chunk for t in done}) > 1


def test_slots_bound_concurrency_and_free_up():
    ds, qs, done, be, srv = run_server(n_slots=2, qps=5000.0, n_q=7)
    assert max(len(a) for kind, _, a in [x for x in be.log if x[0] == "launch"]) <= 2
    # all queries finished although only two fit at a time
    assert len(done) == 7
    # admission waits for a free slot: later queries admitted after earlier ones finished
    adm = sorted(t.admitted for t in done)
    fin = sorted(t.done for t in done)
    assert adm[2] >= fin[0]


def test_memory_budget_limits_admission():
    """The histograms of the queries running together never exceed the
    budget; all queries still finish."""
    qs = datagen.draw_queries(11, 5, qps=5000.0)
    budget = int(1.5 * max(query_hist_bytes(q) for q in qs))
    ds, qs, done, be, srv = run_server(n_slots=4, budget=budget, qps=5000.0, n_q=5)
    assert len(done) == 5
    assert max(be.arena_peak) <= budget // 16
    # fewer queries at once than slots: memory, not slots, was the limit
    launches = [a for kind, _, a in [x for x in be.log if x[0] == "launch"]]
    assert max(len(a) for a in launches) < 4


def test_latency_accounting_and_percentiles():
    ds, qs, done, be, srv = run_server(n_q=12, qps=100.0)
    lat = [t.latency for t in done]
    assert all(l >= be.n_chunks * be.launch_time - 1e-12 for l in lat)
    assert percentile(lat, 50) <= percentile(lat, 99) <= max(lat)
    assert percentile([1.0, 2.0, 3.0, 4.0], 50) == 2.5


def test_closed_loop_runs_all():
    ds = datagen.make_dataset(8, 3000)
    clock = FakeClock()
    be = OracleBackend(ds, 4, 3, clock)
    srv = Server(be, clock=clock, sleep=clock.sleep)
    qs = datagen.draw_queries(3, 5)
    done = srv.run_closed(qs)
    assert sorted(t.qid for t in done) == list(range(5))
    for t in done:
        want = ref.pipeline(ds, [t.query])[0][0]
        assert all(np.array_equal(t.result[h][1], want[h][1]) for h in range(3))


def test_arena_first_fit_and_coalescing():
    a = Arena(100)
    x, y, z = a.alloc(30), a.alloc(30), a.alloc(30)
    assert (x, y, z) == (0, 30, 60) and a.alloc(20) == -1 and a.used() == 90
    a.release(30, 30)
    assert a.alloc(40) == -1          # 30 free in the middle, 10 at the end
    a.release(0, 30)                  # coalesces with [30, 60)
    assert a.alloc(40) == 0 and a.used() == 70
    a.release(0, 40)
    a.release(60, 30)
    assert a.free == [(0, 100)]


def test_budget_is_histogram_memory_and_big_binnings_fit():
    """Histogram memory, not a per-slot reservation, gates admission: with an
    arena a little larger than one 1500-bin query, the queries running
    together never exceed it although eight slots are free; the 1500-bin
    query is admitted once enough memory is free; a query larger than the
    arena is rejected."""
    ds = datagen.make_dataset(9, 4000)
    clock = FakeClock()
    qs = datagen.draw_queries(12, 6, qps=1e6)
    big = datagen.Query(edges_ht=datagen.uniform_edges(1500, 0.0, 3000.0))
    arena = query_slots(big) + 10
    huge = datagen.Query(edges_ht=datagen.uniform_edges(arena, 0.0, 3000.0))
    be = OracleBackend(ds, 4, 8, clock, arena_slots=arena)
    srv = Server(be, clock=clock, sleep=clock.sleep)
    tickets = [srv.submit(q, 0.0) for q in qs + [big, huge]]
    while srv.busy():
        srv.step()
    srv._drain()
    assert max(be.arena_peak) <= arena
    assert tickets[-1].status == "rejected" and tickets[-1].result is None
    done = {t.qid for t in srv.done}
    assert all(t.qid in done for t in tickets[:-1]), "every query that fits the arena finishes"
    want = ref.pipeline(ds, [big])[0][0]
    got = tickets[-2].result
    assert all(np.array_equal(got[h][1], want[h][1]) for h in range(3))
    assert srv.arena.used() == 0


def test_cancel_waiting_and_running_queries():
    ds = datagen.make_dataset(10, 3000)
    clock = FakeClock()
    be = OracleBackend(ds, 5, 1, clock)
    srv = Server(be, clock=clock, sleep=clock.sleep)
    qs = datagen.draw_queries(13, 3)
    a, b, c = (srv.submit(q, 0.0) for q in qs)
    srv.step()
    srv.step()
    assert a.status == "active" and b.status == "pending"
    assert srv.cancel(b) and b.status == "cancelled"
    assert srv.cancel(a) and a.status == "cancelled"
    assert ("clear", a.slot, a.at) in be.log  # its range is zeroed before reuse
    while srv.busy():
        srv.step()
    srv._drain()
    assert [t.qid for t in srv.done] == [c.qid] and c.chunks_seen == 5
    want = ref.pipeline(ds, [c.query])[0][0]
    assert all(np.array_equal(c.result[h][1], want[h][1]) for h in range(3))
    assert not srv.cancel(c) and srv.arena.used() == 0


def test_timeouts_drop_waiting_and_running_queries():
    ds = datagen.make_dataset(11, 3000)
    clock = FakeClock()
    be = OracleBackend(ds, 10, 1, clock, launch_time=0.01)
    srv = Server(be, timeout=0.05, clock=clock, sleep=clock.sleep)
    qs = datagen.draw_queries(14, 2)
    a = srv.submit(qs[0], 0.0)
    b = srv.submit(qs[1], 0.0)
    while srv.busy():
        srv.step()
    srv._drain()
    # a needs 10 passes of 10 ms: it runs past 50 ms and is dropped; b waited
    # behind it for the only slot and expired first or after a short run
    assert a.status == "timeout" and b.status == "timeout"
    assert a.result is None and b.result is None and srv.arena.used() == 0
    assert srv.done == [] and len(srv.dropped) == 2
    # a query with a longer deadline finishes
    c = srv.submit(qs[0], clock(), timeout=1.0)
    while srv.busy():
        srv.step()
    srv._drain()
    assert c.status == "done" and c.chunks_seen == 10


def test_latency_breakdown_adds_up():
    ds, qs, done, be, srv = run_server(n_q=12, qps=100.0)
    for t in done:
        assert t.queue_wait >= 0 and t.scan >= 0 and t.copy_out >= 0
        assert abs(t.queue_wait + t.scan + t.copy_out - t.latency) < 1e-9
