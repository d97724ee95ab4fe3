"""Histogram slots of values at and next to every bin edge, through the fused pass.

The fused kernels take a value's bin from the uniform-bin formula and read
the bin's edges only where the plan has shown the formula can be off (the
bound computed at plan creation from the edges themselves).  Here every event
has one jet and one muon far apart, so H_T and the leading pt of an event are
its jet's pt exactly: the values are put on each edge, on the floats just
below and above it, and between edges, for uniform binnings whose formula is
exact, uniform ones where float32 rounding puts some values one bin off, and
log-spaced ones where it is no guide at all.  The histograms must equal the
oracle's (reading c10: half-open bins, x equal to the last edge overflows).
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd import hepk as H

pytestmark = pytest.mark.gpu


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


def around_edges(edges):
    """Every edge, its float32 neighbours, midpoints, and values beyond both ends."""
    e = np.asarray(edges, np.float32)
    xs = [e, np.nextafter(e, np.float32(-np.inf)), np.nextafter(e, np.float32(np.inf)),
          ((e[:-1].astype(np.float64) + e[1:]) * 0.5).astype(np.float32),
          np.array([e[0] - 1, e[-1] + 1, e[-1] * 2], np.float32)]
    x = np.concatenate(xs)
    return x[x > 0]  # selected jets have pt * s > jet_pt = 0


def one_jet_events(pts, dtype="f32"):
    n = len(pts)
    one = np.ones(n, np.int64)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(one)
    f = np.float32
    jets = datagen.Collection(off.copy(), {"pt": np.asarray(pts, f), "eta": np.zeros(n, f),
                                           "phi": np.zeros(n, f), "mass": np.zeros(n, f)})
    muons = datagen.Collection(off.copy(), {"pt": np.full(n, 50, f), "eta": np.full(n, 1.5, f),
                                            "phi": np.full(n, 3.0, f), "iso": np.zeros(n, f),
                                            "mass": np.zeros(n, f)})
    return datagen.Dataset(n_events=n, jets=jets, muons=muons, weight=np.linspace(0.5, 1.5, n).astype(f))


BINNINGS = {
    "uniform 100 x 20": datagen.uniform_edges(100, 0.0, 2000.0),
    "uniform 100 x 10 (lead)": datagen.uniform_edges(100, 0.0, 1000.0),
    "uniform, offset start": np.linspace(0.1, 1000.7, 101).astype(np.float32),
    "uniform 1000 fine bins": np.linspace(3.0, 503.0, 1001).astype(np.float32),
    "log-spaced": np.geomspace(1.0, 3000.0, 61).astype(np.float32),
    "unit bins": datagen.uniform_edges(21, 0.0, 21.0),
}


@pytest.mark.parametrize("name", list(BINNINGS), ids=list(BINNINGS))
@pytest.mark.parametrize("tune", [None, dict(block=1024), dict(hist_mode=1)], ids=["default", "1024", "global"])
def test_values_at_bin_edges(name, tune):
    edges = BINNINGS[name]
    say(f"bin edges: {name}, tune={tune}")
    x = around_edges(edges)
    ds = one_jet_events(x)
    # H_T binned by the edges under test, the leading pt by the other
    # uniform binning, nJet in unit bins; one scale (single-scale kernels) and
    # three scales around 1 (multi-scale kernels: the values are pt * s)
    queries = [datagen.Query(min_mu=1, min_jet=1, jet_pt=0.0, edges_ht=edges),
               datagen.Query(min_mu=1, min_jet=1, jet_pt=0.0, edges_lead=edges,
                             scales=np.array([1.0, 0.5, 2.0], np.float32))]
    dd = H.DeviceDataset(ds)
    plan = H.Plan([dd], queries, tune)
    s, c = plan.new_hists()
    plan.run(s, c)
    got = plan.split(s, c)[0]
    plan.close()
    want = ref.pipeline(ds, queries)
    for qi, q in enumerate(queries):
        for v in range(q.n_scale):
            for h in range(3):
                gs, gc = got[qi][v][h]
                ws, wc = want[qi][v][h]
                assert np.array_equal(gc.astype(np.uint64), wc.astype(np.uint64)), \
                    f"{name} q{qi} v{v} h{h}: counts differ in slots {np.flatnonzero(gc != wc)[:8]}"
                assert np.all(np.abs(gs - ws) <= 1e-5 * np.abs(ws)), f"{name} q{qi} v{v} h{h}: sumw"
