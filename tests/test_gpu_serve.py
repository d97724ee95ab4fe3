"""Serving on the GPU: each query's histograms are the same alone and in the
mix (co-batched with others, joining the circular scan at any chunk), and
equal the oracle's pass over the whole dataset for that query."""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd import hepk as H
from paper_1906_06242_amd.serve import GpuBackend, Server

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def same(a, b, what):
    for h in range(3):
        assert np.array_equal(a[h][1], b[h][1]), f"counts {what} h{h}"
        assert np.all(np.abs(a[h][0] - b[h][0]) <= RTOL * np.abs(b[h][0])), f"sumw {what} h{h}"


def test_queries_alone_equal_mix_equal_oracle():
    import torch
    assert torch.cuda.is_available()
    H.load()
    say("serve: dataset")
    ds = datagen.make_dataset(21, 150000)
    dd = H.DeviceDataset(ds)
    qs = datagen.draw_queries(9, 10, qps=2000.0)
    say("serve: alone")
    alone = {}
    for i, q in enumerate(qs):
        be = GpuBackend(dd, n_chunks=5, n_slots=1)
        done = Server(be).run_closed([q])
        be.close()
        alone[i] = done[0].result
    say("serve: mix")
    be = GpuBackend(dd, n_chunks=5, n_slots=4)
    srv = Server(be)
    # queries join the circular scan at different chunks while others run
    for q, k in zip(qs, [1, 2, 1, 3, 1, 1, 2, 4, 1, 2]):
        srv.submit(q)
        for _ in range(k):
            srv.step()
    while srv.busy():
        srv.step()
    srv._drain()
    done = srv.done
    be.close()
    assert len(done) == len(qs)
    starts = set()
    for t in done:
        i = next(k for k, q in enumerate(qs) if q is t.query)
        same(t.result, alone[i], f"query {i} mix vs alone")
        same(t.result, ref.pipeline(ds, [t.query])[0][0], f"query {i} vs oracle")
        starts.add(t.start_chunk)
    assert len(starts) > 1
    assert max(t.latency for t in done) > 0


def test_arena_placement_big_binnings_and_cancel():
    """Queries placed in a small histogram arena (memory gates admission), one
    with 1500-bin histograms, one cancelled while running: the others equal
    the oracle, and a query reusing the cancelled one's range starts clean."""
    import torch
    H.load()
    say("serve: arena")
    ds = datagen.make_dataset(22, 60000)
    dd = H.DeviceDataset(ds)
    big = datagen.Query(edges_ht=datagen.uniform_edges(1500, 0.0, 3000.0), jet_pt=35.0)
    qs = datagen.draw_queries(10, 4, qps=2000.0)
    from paper_1906_06242_amd.serve import query_hist_bytes
    budget = query_hist_bytes(big) + 2 * max(query_hist_bytes(q) for q in qs)
    be = GpuBackend(dd, n_chunks=4, n_slots=6, hist_budget=budget, max_bins=1600)
    srv = Server(be)
    tickets = [srv.submit(q) for q in [qs[0], big, qs[1]]]
    srv.step()
    victim = tickets[0]
    assert victim.status == "active" and srv.cancel(victim)
    tickets += [srv.submit(q) for q in qs[2:]]
    while srv.busy():
        srv.step()
    srv._drain()
    be.close()
    assert victim.status == "cancelled"
    for t in tickets[1:]:
        assert t.status == "done", t.status
        same(t.result, ref.pipeline(ds, [t.query])[0][0], f"query {t.qid} vs oracle")
    assert srv.arena.used() == 0
