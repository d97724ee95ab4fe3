"""GPU parity of out-of-core passes (hepk_streamer): a dataset held in host
memory -- pageable, pinned, or memory-mapped from files as the paper's
column cache -- streamed to the device in batches of consecutive events,
with copies overlapping the passes, must give the histograms of the same
pass over the dataset resident in device memory, and of the oracle (counts
exactly, weight sums within a relative 1e-5 per bin)."""
import os
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd import hepk as H

pytestmark = pytest.mark.gpu
RTOL = 1e-5


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    H.load()
    yield
    torch.cuda.synchronize()


def remap(ds, fn):
    """The dataset with every array replaced by fn(name, array)."""
    def coll(name, c):
        if c is None:
            return None
        return datagen.Collection(fn(f"{name}.offsets", c.offsets),
                                  {k: fn(f"{name}.{k}", v) for k, v in c.cols.items()})
    return datagen.Dataset(ds.n_events, coll("jets", ds.jets), coll("muons", ds.muons), fn("weight", ds.weight),
                           coll("electrons", ds.electrons), ds.content_dtype, ds.seed,
                           None if ds.npu is None else fn("npu", ds.npu))


def resident(ds, qs):
    plan = H.Plan([H.DeviceDataset(ds)], qs)
    s, c = plan.new_hists()
    plan.run(s, c)
    out = plan.split(s, c)[0]
    plan.close()
    return out


def streamed(ds, qs, passes=1, **kw):
    import torch
    st = H.Streamer(ds, qs, **kw)
    s, c = st.new_hists()
    for _ in range(passes):
        st.run(s, c)
    torch.cuda.synchronize()
    st.close()
    # the layout is that of a plan over one dataset with these queries
    plan = H.Plan([H.DeviceDataset(datagen.make_dataset(0, 1))], qs)
    out = plan.split(s, c)[0]
    plan.close()
    return out


def check(got, want, qs, times=1, what=""):
    for qi, q in enumerate(qs):
        for v in range(q.n_scale):
            for h in range(3):
                gs, gc = got[qi][v][h]
                ws, wc = want[qi][v][h][:2]
                assert np.array_equal(gc.astype(np.uint64), times * wc.astype(np.uint64)), f"{what} q{qi} v{v} h{h}"
                assert np.all(np.abs(gs - times * ws) <= RTOL * np.abs(times * ws)), f"{what} q{qi} v{v} h{h}"


@pytest.mark.parametrize("batch,bufs", [(7000, 2), (4096, 3), (1 << 22, 2), (1, 1)])
def test_stream_pageable_equals_resident_and_oracle(batch, bufs):
    n = 50000 if batch > 1 else 300
    say(f"stream pageable batch={batch} bufs={bufs} n={n}")
    ds = datagen.make_dataset(80, n)
    qs = [datagen.Query(), datagen.Query(jet_pt=40.0, min_jet=3, scales=datagen.jes_scales()[:4])]
    got = streamed(ds, qs, batch_events=batch, n_buffers=bufs)
    check(got, ref.pipeline(ds, qs), qs, what="vs oracle")
    check(got, resident(ds, qs), qs, what="vs resident")


def test_stream_twice_accumulates():
    say("stream twice")
    ds = datagen.make_dataset(81, 20000)
    qs = [datagen.Query()]
    check(streamed(ds, qs, passes=2, batch_events=3000), ref.pipeline(ds, qs), qs, times=2)


def test_stream_pinned_source():
    say("stream pinned")
    import torch
    ds = datagen.make_dataset(82, 40000)
    pinned = []

    def pin(name, a):
        t = torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        pinned.append(t)
        return t.numpy()
    pds = remap(ds, pin)
    qs = [datagen.Query()]
    check(streamed(pds, qs, batch_events=9000), ref.pipeline(ds, qs), qs)


def test_stream_memory_mapped_cache(tmp_path):
    """Columns saved as uncompressed files and memory-mapped (the column cache
    of Sec. II), then streamed."""
    say("stream memory-mapped")
    ds = datagen.with_pileup(datagen.make_dataset(83, 30000, extended=True, content_dtype="f16"), 83)

    def to_file(name, a):
        path = os.path.join(tmp_path, name + ".npy")
        np.save(path, np.ascontiguousarray(a))
        return np.load(path, mmap_mode="r")
    mds = remap(ds, to_file)
    qs = [datagen.lookup_query(), datagen.extended_query()]
    got = streamed(mds, qs, batch_events=8192, n_buffers=2, host_threads=4)
    check(got, ref.pipeline(ds, qs), qs)


def test_stream_empty_dataset():
    say("stream empty")
    ds = datagen.make_dataset(84, 0)
    qs = [datagen.Query()]
    got = streamed(ds, qs, batch_events=100)
    for h in range(3):
        assert got[0][0][h][1].sum() == 0
