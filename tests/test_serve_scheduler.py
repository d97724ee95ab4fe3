"""The serving scheduler on the CPU: the oracle as the device, a fake clock.

Checks continuous batching: queries are admitted as slots and histogram
memory free up, every query sees every chunk exactly once whatever chunk it
starts at, results equal the oracle's full pass for that query alone, and
latency bookkeeping follows the clock.
"""
import numpy as np

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd.serve import Server, percentile, query_hist_bytes


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

    def __init__(self, ds, n_chunks, n_slots, clock, launch_time=0.001):
        n = ds.n_events
        b = [n * c // n_chunks for c in range(n_chunks + 1)]
        self.chunks = [host_slice(ds, b[c], b[c + 1]) for c in range(n_chunks)]
        self.n_chunks, self.n_slots = n_chunks, n_slots
        self.q = [None] * n_slots
        self.h = [None] * n_slots
        self.clock, self.launch_time = clock, launch_time
        self.log = []

    def set_query(self, slot, q):
        self.q[slot] = q
        if q is not None:
            self.h[slot] = [(np.zeros(len(e) + 1), np.zeros(len(e) + 1, np.uint64)) for e in q.edges()]
        self.log.append(("set", slot, q is not None))

    def launch(self, c):
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

    def snapshot_and_clear(self, slot, q):
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
    be = OracleBackend(ds, C, n_slots, clock)
    srv = Server(be, hist_budget=budget, clock=clock, sleep=clock.sleep)
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
    q = datagen.Query()
    one = query_hist_bytes(q)
    ds, qs, done, be, srv = run_server(n_slots=4, budget=int(1.5 * query_hist_bytes(datagen.draw_queries(11, 1)[0])),
                                       qps=5000.0, n_q=5)
    assert len(done) == 5
    launches = [a for kind, _, a in [x for x in be.log if x[0] == "launch"]]
    # query histograms here are 50-200 bins: at most 2 fit in 1.5 x the first one's bytes
    assert max(len(a) for a in launches) <= 2
    assert one > 0


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
