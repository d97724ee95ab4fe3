"""hepk_pipeline_noalloc (the fused pass with its tables in the library's
fixed device array) against hepk_plan_create + hepk_pipeline: the same
histograms, on two calls in a row whose second input is smaller, for the
single-scale and the 20-scale extended pass; tables beyond the fixed array
are rejected before anything runs."""
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


class Layout:
    """The histogram layout of a closed plan: slot count and block offsets."""

    def __init__(self, plan, qs):
        self.n_slots = plan.n_slots
        self.off = {(d, qi, v, h): plan.hist_offset(d, qi, v, h)
                    for d in range(len(plan.datasets)) for qi, q in enumerate(qs)
                    for v in range(q.n_scale) for h in range(3)}

    def hist_offset(self, d, qi, v, h):
        return self.off[(d, qi, v, h)]


def planned(dds, qs, tune=None):
    plan = H.Plan(dds, qs, tune)
    s, c = plan.new_hists()
    plan.run(s, c)
    out = (s.cpu().numpy(), c.cpu().numpy())
    lay = Layout(plan, qs)
    plan.close()
    return out, lay


def noalloc(dds, qs, n_slots, tune=None):
    import torch
    s = torch.zeros(n_slots, dtype=torch.float64, device="cuda")
    c = torch.zeros(n_slots, dtype=torch.int64, device="cuda")
    H.pipeline_noalloc(dds, qs, s, c, tune)
    return s.cpu().numpy(), c.cpu().numpy()


def check(got, want, what):
    gs, gc = got
    ws, wc = want
    assert np.array_equal(gc, wc), f"counts {what}"
    assert np.all(np.abs(gs - ws) <= 1e-5 * np.abs(ws)), f"sumw {what}"


@pytest.mark.parametrize("extended", [False, True])
def test_noalloc_equals_plan_twice(extended):
    for n in (30011, 1234):  # the second call has a smaller input
        say(f"noalloc extended={extended} n={n}")
        if extended:
            ds = datagen.make_dataset(5, n, extended=True, content_dtype="f16")
            qs = [datagen.extended_query()]
        else:
            ds = datagen.make_dataset(5, n)
            qs = [datagen.Query(), datagen.Query(mu_pt=25.0, jet_pt=40.0, min_jet=3)]
        dds = [H.DeviceDataset(ds)]
        want, plan = planned(dds, qs)
        got = noalloc(dds, qs, plan.n_slots)
        check(got, want, f"n={n}")
        # and the oracle agrees on the first query's histograms
        o = ref.pipeline(ds, qs[:1])[0]
        for v in range(qs[0].n_scale):
            for h in range(3):
                off = plan.hist_offset(0, 0, v, h)
                sl = slice(off[0], off[0] + off[1] + 2)
                check((got[0][sl], got[1][sl].view(np.uint64)), o[v][h], f"oracle v={v} h={h}")


def test_noalloc_batch_and_tune():
    say("noalloc batch")
    sizes = [0, 700, 5000, 64, 12345]
    dss = [datagen.make_dataset(40 + i, n) for i, n in enumerate(sizes)]
    dds = [H.DeviceDataset(d) for d in dss]
    qs = [datagen.Query()]
    for tune in (None, {"block": 256, "ev_per_thread": 2, "hist_mode": 1}):
        want, plan = planned(dds, qs, tune)
        check(noalloc(dds, qs, plan.n_slots, tune), want, f"batch tune={tune}")


def test_noalloc_rejects_tables_beyond_its_array():
    say("noalloc too large")
    import torch
    ds = datagen.make_dataset(6, 100)
    dds = [H.DeviceDataset(ds)] * 8000  # 8000 dataset entries (176 B each): beyond 1 MiB of tables
    s = torch.zeros(1, dtype=torch.float64, device="cuda")
    c = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(H.HepkError) as ei:
        H.pipeline_noalloc(dds, [datagen.Query()], s, c)
    assert ei.value.status == H.EINVAL
    assert "fixed scratch" in str(ei.value)
