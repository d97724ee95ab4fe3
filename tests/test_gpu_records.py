"""Per-event parity of the fused pass.

hepk_pipeline_debug runs the fused kernels with per-event record stores and
returns, for every event and jet-energy scale, the selected-muon count, the
selected and b-tagged jet counts, H_T, the leading pt and whether the event
passed.  Each is compared bit for bit (float32 as uint32) with the same
values composed from the oracle's primitives (ref.pipeline_events), for every
launch shape of the single-scale and multi-scale kernels, base and extended
schemas, float32 and float16 content, non-finite content (reading c9: NaN
fails every cut and never becomes a minimum), and tiles beyond the on-chip
capacity.  Events the kernel proves unable to pass before walking their jets
must be exactly those with a documented reason, and none of them may pass in
the oracle.
"""
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


def u32(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def with_nonfinite(ds, seed):
    """NaN and +-inf in a few hundred jet, muon and electron pt/eta/phi/iso
    entries (weights stay finite)."""
    rng = np.random.default_rng(seed)
    bad = np.array([np.nan, np.inf, -np.inf], np.float32)
    for _, coll in ds.collections():
        for k, col in coll.cols.items():
            if k == "mass" or col.size == 0:
                continue
            idx = rng.integers(0, col.size, max(1, col.size // 300))
            col[idx] = bad[rng.integers(0, 3, idx.size)].astype(col.dtype)
    return ds


def with_dense_runs(ds, seed):
    """Runs of events with many objects (12 and 20 jets, 5 muons, 4
    electrons) so tiles exceed the on-chip capacity and run as sub-tiles, and
    two single events beyond it (one lane, straight from HBM)."""
    rng = np.random.default_rng(seed)
    jc = np.diff(ds.jets.offsets).copy()
    mc = np.diff(ds.muons.offsets).copy()
    jc[1000:1300] = 12
    jc[1500:1600] = 20
    mc[2000:2200] = 5
    jc[2500], mc[2500] = 1500, 3
    jc[2501], mc[2501] = 30, 400

    def rebuild(coll, counts):
        off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
        return datagen.Collection(off, {k: rng.choice(v, int(off[-1])).astype(v.dtype) for k, v in coll.cols.items()})

    els = None
    if ds.electrons is not None:
        ec = np.diff(ds.electrons.offsets).copy()
        ec[2700:2900] = 4
        ec[2502] = 300
        els = rebuild(ds.electrons, ec)
    return datagen.Dataset(ds.n_events, rebuild(ds.jets, jc), rebuild(ds.muons, mc), ds.weight, els,
                           ds.content_dtype)


def skip_reasons(ds, q, want, ms):
    """Events the fused kernel may leave unwalked: too few selected muons,
    too few jets before any cut, or (plans with several scales, jet_pt >= 0)
    too few selected or b-tagged jets at the query's largest scale."""
    nj_all = np.diff(ds.jets.offsets)
    r = (want[0]["n_mu"] < q.min_mu) | (nj_all < q.min_jet)
    if ms and q.jet_pt >= 0:
        smax = np.float32(np.max(q.scales))
        top = ref.pipeline_events(ds, datagen.Query(**{**q.__dict__, "scales": np.array([smax], np.float32)}))[0]
        r |= (top["n_jet"] < q.min_jet)
        if "btag" in ds.jets.cols:
            r |= (top["n_b"] < q.min_b)
    return r


def check_records(ds, queries, tune=None, what=""):
    dd = H.DeviceDataset(ds)
    plan = H.Plan([dd], queries, tune)
    ms = any(q.n_scale > 1 for q in queries)
    s, c = plan.new_hists()
    rec = plan.run_debug(s, c)[0]
    got_h = plan.split(s, c)[0]
    plan.close()
    want_h = ref.pipeline(ds, queries)
    n_walked = 0
    for qi, q in enumerate(queries):
        want = ref.pipeline_events(ds, q)
        reasons = skip_reasons(ds, q, want, ms)
        for v in range(q.n_scale):
            r, w = rec[qi][v], want[v]
            tag = f"{what} q{qi} v{v}"
            st = r["state"]
            assert np.all((st >= 1) & (st <= 3)), f"{tag}: {int(np.sum(st < 1))} records not written"
            assert np.array_equal(r["n_mu"], w["n_mu"]), f"{tag}: n_mu"
            assert np.array_equal(u32(r["w"]), u32(w["weight"])), f"{tag}: event weight"
            walked = st >= 2
            n_walked += int(walked.sum())
            for f in ("n_jet", "n_b"):
                bad = np.flatnonzero(r[f][walked] != w[f][walked])
                assert bad.size == 0, f"{tag}: {f} differs at {np.flatnonzero(walked)[bad[:5]]}"
            for f in ("ht", "lead"):
                bad = np.flatnonzero(u32(r[f][walked]) != u32(w[f][walked]))
                assert bad.size == 0, f"{tag}: {f} bits differ at {np.flatnonzero(walked)[bad[:5]]}"
            assert np.array_equal(st[walked] == 3, w["passed"][walked] == 1), f"{tag}: pass"
            skipped = ~walked
            assert not np.any(w["passed"][skipped]), f"{tag}: an unwalked event passes in the oracle"
            assert np.all(reasons[skipped]), f"{tag}: an event left unwalked without a reason"
            assert np.all(r["n_jet"][skipped] == 0) and np.all(r["n_b"][skipped] == 0)
            assert np.all(u32(r["ht"][skipped]) == 0) and np.all(np.isneginf(r["lead"][skipped]))
            for h in range(3):
                gs, gc = got_h[qi][v][h]
                ws, wc = want_h[qi][v][h]
                assert np.array_equal(gc.astype(np.uint64), wc.astype(np.uint64)), f"{tag} h{h} counts"
                assert np.all(np.abs(gs - ws) <= RTOL * np.abs(ws)), f"{tag} h{h} sumw"
    assert n_walked > 0
    return rec


TUNES = [None, dict(block=512), dict(ev_per_thread=2), dict(block=512, ev_per_thread=2),
         dict(block=256), dict(block=256, ev_per_thread=2), dict(hist_mode=1), dict(grid=7),
         dict(block=1024), dict(block=1024, hist_mode=1, grid=3)]


def single_scale_queries(extended):
    return [datagen.Query(min_b=1 if extended else 0),
            datagen.Query(jet_pt=-1.0, min_mu=0, min_jet=2),       # no zero-store shortcut
            datagen.Query(mu_pt=25.0, jet_pt=40.0, min_jet=3, dr=0.0),
            datagen.Query(min_mu=0, min_jet=0, scales=np.array([0.97], np.float32))]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("tune", TUNES, ids=[str(t) for t in TUNES])
def test_records_single_scale(tune, extended, dtype):
    say(f"records single-scale tune={tune} extended={extended} dtype={dtype}")
    ds = with_nonfinite(datagen.make_dataset(40, 20000, extended=extended, content_dtype=dtype), 1)
    check_records(ds, single_scale_queries(extended), tune, f"single {tune} {dtype}")


MS_TUNES = [None, dict(block=256), dict(ev_per_thread=2), dict(block=256, ev_per_thread=2), dict(block=512),
            dict(hist_mode=1), dict(block=1024), dict(block=1024, hist_mode=1)]


def mixed_queries(extended):
    sc = datagen.jes_scales()
    return [datagen.Query(),
            datagen.Query(min_b=1 if extended else 0, scales=sc[:3]),
            datagen.Query(jet_pt=25.0, min_jet=2, scales=sc[:5]),
            datagen.Query(min_b=1 if extended else 0, scales=sc),
            datagen.Query(jet_pt=-1.0, min_jet=6, scales=sc[5:11]),
            datagen.Query(min_mu=0, min_jet=0, scales=sc[12:19])]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("tune", MS_TUNES, ids=[str(t) for t in MS_TUNES])
def test_records_several_scales(tune, extended, dtype):
    say(f"records several scales tune={tune} extended={extended} dtype={dtype}")
    ds = with_nonfinite(datagen.make_dataset(41, 12000, extended=extended, content_dtype=dtype), 2)
    check_records(ds, mixed_queries(extended), tune, f"multi {tune} {dtype}")


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("extended", [False, True])
def test_records_dense_and_oversized_tiles(extended, dtype):
    base = datagen.make_dataset(42, 4000, extended=extended, content_dtype=dtype)
    ds = with_dense_runs(with_nonfinite(base, 3), 4)
    for tune in (None, dict(block=256, ev_per_thread=2), dict(block=512, ev_per_thread=2, hist_mode=1),
                 dict(block=1024)):
        say(f"records dense tiles tune={tune} extended={extended} dtype={dtype}")
        check_records(ds, single_scale_queries(extended), tune, f"dense single {tune}")
        check_records(ds, mixed_queries(extended)[:4], tune, f"dense multi {tune}")


def test_records_batch_of_datasets():
    """Records of several datasets in one launch land at each dataset's
    place, every dataset equal to the oracle on its own."""
    say("records batch")
    sizes = [0, 1, 257, 9000, 64]
    dss = [with_nonfinite(datagen.make_dataset(50 + i, n), 5 + i) for i, n in enumerate(sizes)]
    qs = [datagen.Query(), datagen.Query(jet_pt=35.0, min_jet=3, scales=datagen.jes_scales()[:6])]
    plan = H.Plan([H.DeviceDataset(d) for d in dss], qs, dict(grid=5))
    s, c = plan.new_hists()
    rec = plan.run_debug(s, c)
    plan.close()
    for d, ds in enumerate(dss):
        for qi, q in enumerate(qs):
            want = ref.pipeline_events(ds, q)
            for v in range(q.n_scale):
                r = rec[d][qi][v]
                assert len(r) == ds.n_events
                assert np.array_equal(r["n_mu"], want[v]["n_mu"]), f"d{d} q{qi} v{v}"
                walked = r["state"] >= 2
                assert np.array_equal(u32(r["ht"][walked]), u32(want[v]["ht"][walked])), f"d{d} q{qi} v{v}"
                assert np.array_equal((r["state"] == 3), want[v]["passed"] == 1), f"d{d} q{qi} v{v}"


def test_records_full_size_1e7():
    """The benchmark workload (1e7 events, default launch configuration):
    every event's record equal to the oracle's values."""
    say("records full size 1e7")
    ds = datagen.make_dataset(0, 10_000_000)
    check_records(ds, [datagen.Query()], None, "1e7")
