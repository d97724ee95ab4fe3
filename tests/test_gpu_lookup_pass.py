"""GPU parity of the fused pass with lookup corrections (Sec. IV: event
weights from pileup and lepton scale-factor lookups, jet energies shifted by
an interpolated uncertainty table) and sums of squared weights.

Per event and scale, the fused kernel's records (selected muons, selected
and b-tagged jets, H_T, leading pt, pass, event weight) are compared bit for
bit with the values composed from the oracle's primitives
(ref.pipeline_events); the histograms with ref.pipeline (counts exactly,
float64 sums and squared-weight sums within a relative 1e-5 per bin).
Single-scale and several-scale plans, factor and shift scales, base and
extended schemas, float32 and float16, non-finite content, oversized tiles
and every launch shape of the lookup kernels are covered.
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_1906_06242_amd import datagen
from paper_1906_06242_amd import hepk as H

import test_gpu_records as R

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


u32 = R.u32
PU, SF, JES = datagen.pileup_table(), datagen.muon_sf_table(), datagen.jes_table()
SHIFTS = datagen.jes_lookup_shifts()


def single_scale_queries(extended):
    mb = 1 if extended else 0
    return [datagen.Query(pu=PU, sf=SF, min_b=mb),                                   # factor 1, weights
            datagen.Query(pu=PU, sf=SF, jes=JES, scales=np.array([0.0], np.float32), min_b=mb),
            datagen.Query(jes=JES, scales=np.array([1.5], np.float32), jet_pt=-1.0, min_mu=0, min_jet=2),
            datagen.Query(sf=SF, jes=JES, scales=np.array([-2.0], np.float32), jet_pt=45.0, min_jet=3)]


def several_scale_queries(extended):
    mb = 1 if extended else 0
    return [datagen.Query(pu=PU, sf=SF, jes=JES, scales=SHIFTS, min_b=mb),
            datagen.Query(pu=PU, jes=JES, scales=SHIFTS[:5], jet_pt=-1.0, min_jet=3),
            datagen.Query(pu=PU, scales=datagen.jes_scales()[:4], min_b=mb),
            datagen.Query(sf=SF, jes=JES, scales=np.array([-40.0, 25.0, 0.0], np.float32), min_mu=0, min_jet=2)]


def check_lookup_pass(ds, queries, tune=None, what=""):
    dd = H.DeviceDataset(ds)
    plan = H.Plan([dd], queries, tune)
    s, c = plan.new_hists()
    rec = plan.run_debug(s, c)[0]
    got_h = plan.split(s, c)[0]
    # the squared weights from a second pass (same kernels, same histograms)
    s2, c2 = plan.new_hists()
    w2 = s2.clone()
    plan.run_w2(s2, w2, c2)
    got_w2 = plan.split(w2, c2)[0]
    got_h2 = plan.split(s2, c2)[0]
    plan.close()
    want_h = ref.pipeline(ds, queries, want_sumw2=True)
    n_walked = 0
    for qi, q in enumerate(queries):
        want = ref.pipeline_events(ds, q)
        for v in range(q.n_scale):
            r, w = rec[qi][v], want[v]
            tag = f"{what} q{qi} v{v}"
            st = r["state"]
            assert np.all((st >= 1) & (st <= 3)), f"{tag}: records not written"
            assert np.array_equal(r["n_mu"], w["n_mu"]), f"{tag}: n_mu"
            bad = np.flatnonzero(u32(r["w"]) != u32(w["weight"]))
            assert bad.size == 0, f"{tag}: weight bits differ at {bad[:5]}"
            walked = st >= 2
            n_walked += int(walked.sum())
            for f in ("n_jet", "n_b"):
                bad = np.flatnonzero(r[f][walked] != w[f][walked])
                assert bad.size == 0, f"{tag}: {f} differs at {np.flatnonzero(walked)[bad[:5]]}"
            for f in ("ht", "lead"):
                bad = np.flatnonzero(u32(r[f][walked]) != u32(w[f][walked]))
                assert bad.size == 0, f"{tag}: {f} bits differ at {np.flatnonzero(walked)[bad[:5]]}"
            assert np.array_equal(st[walked] == 3, w["passed"][walked] == 1), f"{tag}: pass"
            assert not np.any(w["passed"][~walked]), f"{tag}: an unwalked event passes in the oracle"
            for h in range(3):
                ws, wc, ww2 = want_h[qi][v][h]
                for name, (gs, gc) in (("debug", got_h[qi][v][h]), ("w2 pass", got_h2[qi][v][h])):
                    assert np.array_equal(gc.astype(np.uint64), wc.astype(np.uint64)), f"{tag} h{h} {name} counts"
                    assert np.all(np.abs(gs - ws) <= RTOL * np.abs(ws)), f"{tag} h{h} {name} sumw"
                g2 = got_w2[qi][v][h][0]
                assert np.all(np.abs(g2 - ww2) <= RTOL * np.abs(ww2)), f"{tag} h{h} sumw2"
    assert n_walked > 0


LK_TUNES = [None, dict(block=256), dict(block=512), dict(block=1024), dict(hist_mode=1), dict(grid=7),
            dict(block=256, ev_per_thread=2)]


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("tune", LK_TUNES, ids=[str(t) for t in LK_TUNES])
def test_lookup_pass_single_scale(tune, extended, dtype):
    say(f"lookup pass single-scale tune={tune} extended={extended} dtype={dtype}")
    ds = R.with_nonfinite(datagen.make_dataset(60, 15000, extended=extended, content_dtype=dtype), 7)
    check_lookup_pass(datagen.with_pileup(ds, 60), single_scale_queries(extended), tune, f"single {tune}")


@pytest.mark.parametrize("dtype", ["f32", "f16"])
@pytest.mark.parametrize("extended", [False, True])
@pytest.mark.parametrize("tune", LK_TUNES, ids=[str(t) for t in LK_TUNES])
def test_lookup_pass_several_scales(tune, extended, dtype):
    say(f"lookup pass several scales tune={tune} extended={extended} dtype={dtype}")
    ds = R.with_nonfinite(datagen.make_dataset(61, 9000, extended=extended, content_dtype=dtype), 8)
    check_lookup_pass(datagen.with_pileup(ds, 61), several_scale_queries(extended), tune, f"multi {tune}")


@pytest.mark.parametrize("extended", [False, True])
def test_lookup_pass_dense_and_oversized_tiles(extended):
    base = datagen.make_dataset(62, 4000, extended=extended, content_dtype="f16" if extended else "f32")
    ds = datagen.with_pileup(R.with_dense_runs(R.with_nonfinite(base, 9), 10), 62)
    for tune in (None, dict(block=256), dict(block=1024, hist_mode=1)):
        say(f"lookup pass dense tiles tune={tune} extended={extended}")
        check_lookup_pass(ds, single_scale_queries(extended), tune, f"dense single {tune}")
        check_lookup_pass(ds, several_scale_queries(extended)[:2], tune, f"dense multi {tune}")


def test_lookup_pass_without_pileup_column():
    """A pileup table on a dataset without a pileup column: that factor is
    not applied (the oracle does the same)."""
    say("lookup pass without npu")
    ds = datagen.make_dataset(63, 7000)
    check_lookup_pass(ds, single_scale_queries(False)[:2], None, "no npu")


def test_lookup_pass_factor_one_equals_plain_pass():
    """Lookup tables of constant 1 and zero shifts reproduce the plain pass."""
    say("lookup pass reduces to the plain pass")
    ds = datagen.with_pileup(datagen.make_dataset(64, 20000), 64)
    pe, pc = PU
    se, sc = SF
    ee, pt_e, d = JES
    ones = datagen.Query(pu=(pe, np.ones_like(pc)), sf=(se, np.ones_like(sc)), jes=(ee, pt_e, d),
                         scales=np.array([0.0], np.float32))
    dd = H.DeviceDataset(ds)
    got = []
    for q in (ones, datagen.Query()):
        plan = H.Plan([dd], [q])
        s, c = plan.new_hists()
        plan.run(s, c)
        got.append(plan.split(s, c)[0][0][0])
        plan.close()
    for h in range(3):
        assert np.array_equal(got[0][h][1], got[1][h][1])
        assert np.array_equal(got[0][h][0], got[1][h][0])


def test_sumw2_plain_plan():
    """opts.sumw2 on a plan without lookups: the plain pass plus squared
    weights, equal to the oracle's."""
    say("sumw2 plain plan")
    import torch
    ds = datagen.make_dataset(65, 30000)
    qs = [datagen.Query(), datagen.Query(scales=datagen.jes_scales()[:3], jet_pt=35.0)]
    for q in qs:
        plan = H.Plan([H.DeviceDataset(ds)], [q], sumw2=True)
        s, c = plan.new_hists()
        w2 = torch.zeros_like(s)
        plan.run_w2(s, w2, c)
        got_s, got_w2 = plan.split(s, c)[0][0], plan.split(w2, c)[0][0]
        plan.close()
        want = ref.pipeline(ds, [q], want_sumw2=True)[0]
        for v in range(q.n_scale):
            for h in range(3):
                ws, wc, ww2 = want[v][h]
                assert np.array_equal(got_s[v][h][1].astype(np.uint64), wc.astype(np.uint64))
                assert np.all(np.abs(got_s[v][h][0] - ws) <= RTOL * np.abs(ws))
                assert np.all(np.abs(got_w2[v][h][0] - ww2) <= RTOL * np.abs(ww2))


def test_w2_needs_a_lookup_plan():
    say("w2 refused on a plain plan")
    import torch
    ds = datagen.make_dataset(66, 100)
    plan = H.Plan([H.DeviceDataset(ds)], [datagen.Query()])
    s, c = plan.new_hists()
    with pytest.raises(H.HepkError) as ei:
        plan.run_w2(s, torch.zeros_like(s), c)
    assert ei.value.status == H.EINVAL
    plan.close()


def test_lookup_queries_are_not_installed_in_slots():
    say("set_query refuses lookup queries")
    ds = datagen.make_dataset(67, 100)
    plan = H.Plan([H.DeviceDataset(ds)], [datagen.Query()], reserve_bins=200)
    with pytest.raises(H.HepkError) as ei:
        plan.set_query(0, datagen.Query(pu=PU))
    assert ei.value.status == H.EUNSUPPORTED
    plan.close()
