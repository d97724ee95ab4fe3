"""GPU parity of the lookup primitives against the CPU oracle.

hepk_get_bin_contents, hepk_interp and hepk_jes_delta must equal the oracle
bit for bit (a NaN result only needs to be NaN on both sides); the PROD
reduction bit for bit; the squared-weight fill's counts exactly and its
float64 sums within a relative 1e-5 per bin.  Inputs cover exact edges and
bin centres, values beyond both ends, NaN and infinities, float16 and int32
columns, unaligned views (the row-by-row kernels), tables too large for LDS
(read from HBM) and single-bin tables.
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


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def assert_same_f32(got, want, what):
    got, want = np.asarray(got, np.float32), np.asarray(want, np.float32)
    assert got.shape == want.shape, what
    both_nan = np.isnan(got) & np.isnan(want)
    same = (got.view(np.uint32) == want.view(np.uint32)) | both_nan
    if not np.all(same):
        i = int(np.flatnonzero(~same)[0])
        raise AssertionError(f"{what}: {np.count_nonzero(~same)} differ, first at {i}: {got[i]!r} vs {want[i]!r}")


def table(rng, nbins, uniform=True, lo=-3.0, hi=5.0):
    if uniform:
        edges = datagen.uniform_edges(nbins, lo, hi)
    else:
        pool = np.unique(rng.uniform(lo, hi, 4 * (nbins + 1)).astype(np.float32))
        edges = np.sort(rng.choice(pool, nbins + 1, replace=False))
    contents = rng.normal(1.0, 0.3, len(edges) + 1).astype(np.float32)
    return np.ascontiguousarray(edges, np.float32), contents


def probe_values(rng, edges, n):
    """Values at edges, at bin centres, just beside them, beyond both ends,
    non-finite, and uniform over the range; n in total."""
    e = edges.astype(np.float32)
    c = ((e[:-1] + e[1:]) * np.float32(0.5)).astype(np.float32)
    special = np.concatenate([
        e, c, np.nextafter(e, np.float32(-np.inf)), np.nextafter(c, np.float32(np.inf)),
        np.nextafter(c, np.float32(-np.inf)),
        np.array([np.nan, np.inf, -np.inf, e[0] - 10, e[-1] + 10, 0.0, -0.0], np.float32)]).astype(np.float32)
    span = float(e[-1] - e[0])
    body = rng.uniform(float(e[0]) - 0.1 * span, float(e[-1]) + 0.1 * span, max(0, n - len(special)))
    x = np.concatenate([special, body.astype(np.float32)])[:n]
    rng.shuffle(x)
    return np.ascontiguousarray(x, np.float32)


@pytest.mark.parametrize("n", [0, 1, 5, 1023, 100003])
@pytest.mark.parametrize("nbins,uniform", [(1, True), (7, False), (100, True), (7000, False)])
def test_get_bin_contents_and_interp(n, nbins, uniform):
    say(f"lookup n={n} nbins={nbins} uniform={uniform}")
    rng = np.random.default_rng(1000 * nbins + n)
    edges, contents = table(rng, nbins, uniform)
    x = probe_values(rng, edges, n) if n > 0 else np.zeros(0, np.float32)
    de, dc = dev(edges), dev(contents)
    for name, g, w in (("get_bin_contents", H.get_bin_contents, ref.get_bin_contents),
                       ("interp", H.interp, ref.interp)):
        want = w(x, edges, contents)
        got = g(dev(x), de, dc).cpu().numpy()
        assert_same_f32(got, want, f"{name} n={n} nbins={nbins}")
        if n > 1:
            # an unaligned view takes the row-by-row kernel
            import torch
            big = dev(np.concatenate([[np.float32(0)], x]))
            got = g(big[1:], de, dc).cpu().numpy()
            assert_same_f32(got, w(x, edges, contents), f"{name} unaligned n={n}")


@pytest.mark.parametrize("dtype", ["f16", "i32"])
def test_lookup_other_dtypes(dtype):
    say(f"lookup dtype={dtype}")
    rng = np.random.default_rng(7)
    edges, contents = table(rng, 40, True, lo=-20.0, hi=20.0)
    if dtype == "f16":
        x = probe_values(rng, edges, 5003).astype(np.float16)
    else:
        x = rng.integers(-30, 31, 5003).astype(np.int32)
    for g, w in ((H.get_bin_contents, ref.get_bin_contents), (H.interp, ref.interp)):
        assert_same_f32(g(dev(x), dev(edges), dev(contents)).cpu().numpy(), w(x, edges, contents), f"{dtype}")


def test_lookup_tables_of_the_analysis():
    """The synthetic pileup and muon scale-factor tables on analysis-like inputs."""
    say("lookup analysis tables")
    ds = datagen.with_pileup(datagen.make_dataset(3, 50000), 3)
    pe, pc = datagen.pileup_table()
    se, sc = datagen.muon_sf_table()
    assert_same_f32(H.get_bin_contents(dev(ds.npu), dev(pe), dev(pc)).cpu().numpy(),
                    ref.get_bin_contents(ds.npu, pe, pc), "pileup")
    mpt = ds.muons.cols["pt"]
    assert_same_f32(H.get_bin_contents(dev(mpt), dev(se), dev(sc)).cpu().numpy(),
                    ref.get_bin_contents(mpt, se, sc), "muon sf")
    assert_same_f32(H.interp(dev(mpt), dev(se), dev(sc)).cpu().numpy(), ref.interp(mpt, se, sc), "muon sf interp")


def test_lookups_several_grid_steps():
    """2e7 + 3 rows: more rows than one grid step covers (16 workgroups per
    CU for the one-dimensional lookups, 64 for the shift), so every kernel
    walks several steps, the last one partial; bits equal to the oracle's."""
    say("lookups several grid steps")
    rng = np.random.default_rng(91)
    n = 20_000_003
    pe, pc = datagen.pileup_table()
    se, sc = datagen.muon_sf_table()
    ee, pte, d = datagen.jes_table()
    x = rng.uniform(0.0, 200.0, n).astype(np.float32)
    h = rng.uniform(-5.0, 5.0, n).astype(np.float32)
    dx = dev(x)
    assert_same_f32(H.get_bin_contents(dx, dev(pe), dev(pc)).cpu().numpy(), ref.get_bin_contents(x, pe, pc),
                    "contents")
    assert_same_f32(H.interp(dx, dev(se), dev(sc)).cpu().numpy(), ref.interp(x, se, sc), "interp")
    assert_same_f32(H.jes_delta(dx, dev(h), dev(ee), dev(pte), dev(d)).cpu().numpy(),
                    ref.jes_delta(x, h, ee, pte, d), "jes shift")


@pytest.mark.parametrize("n", [0, 3, 4099, 200001])
@pytest.mark.parametrize("content", ["f32", "f16"])
def test_jes_delta(n, content):
    say(f"jes_delta n={n} {content}")
    rng = np.random.default_rng(n + 17)
    ee, pe, d = datagen.jes_table()
    pt = (20.0 + rng.exponential(60.0, n)).astype(np.float32)
    eta = rng.normal(0.0, 2.0, n).astype(np.float32)
    if n > 64:
        c = ((pe[:-1] + pe[1:]) * np.float32(0.5)).astype(np.float32)
        pt[:len(c)] = c
        pt[len(c):len(c) + len(pe)] = pe
        pt[-6:] = [np.nan, np.inf, -np.inf, 1.0, 5000.0, 0.0]
        eta[:len(ee)] = ee
        eta[len(ee):2 * len(ee)] = -ee
        eta[-12:-6] = [np.nan, np.inf, -np.inf, 4.7, -4.7, 0.0]
    if content == "f16":
        pt, eta = pt.astype(np.float16), eta.astype(np.float16)
    want = ref.jes_delta(pt, eta, ee, pe, d)
    got = H.jes_delta(dev(pt), dev(eta), dev(ee), dev(pe), dev(d)).cpu().numpy()
    assert_same_f32(got, want, f"jes_delta n={n}")
    if n > 1:
        # unaligned views
        got = H.jes_delta(dev(np.concatenate([pt[:1], pt]))[1:], dev(np.concatenate([eta[:1], eta]))[1:],
                          dev(ee), dev(pe), dev(d)).cpu().numpy()
        assert_same_f32(got, want, f"jes_delta unaligned n={n}")


def test_jes_delta_large_table():
    """A table too large for LDS is read from HBM; same results."""
    say("jes_delta large table")
    rng = np.random.default_rng(5)
    ee = np.sort(np.unique(rng.uniform(0, 5, 130).astype(np.float32)))[:101]
    pe = np.sort(np.unique(rng.uniform(10, 2000, 200).astype(np.float32)))[:151]
    d = rng.normal(0.03, 0.01, (len(ee) - 1, len(pe) - 1)).astype(np.float32)
    pt = rng.uniform(0, 2100, 30011).astype(np.float32)
    eta = rng.uniform(-5.5, 5.5, 30011).astype(np.float32)
    assert_same_f32(H.jes_delta(dev(pt), dev(eta), dev(ee), dev(pe), dev(d)).cpu().numpy(),
                    ref.jes_delta(pt, eta, ee, pe, d), "large table")


@pytest.mark.parametrize("n_events", [0, 1, 1000, 70001])
def test_reduce_prod(n_events):
    say(f"reduce PROD n={n_events}")
    ds = datagen.make_dataset(11, n_events) if n_events else None
    if ds is None:
        off = np.zeros(1, np.int64)
        content = np.zeros(0, np.float32)
    else:
        off = ds.muons.offsets
        se, sc = datagen.muon_sf_table()
        content = ref.get_bin_contents(ds.muons.cols["pt"], se, sc)
    rng = np.random.default_rng(n_events)
    m = (rng.uniform(size=len(content)) < 0.7).astype(np.uint8)
    em = (rng.uniform(size=n_events) < 0.9).astype(np.uint8)
    # a device column of no objects still needs a valid pointer (one unused element)
    dcontent = dev(content if content.size else np.zeros(1, np.float32))
    for om in (None, m):
        for evm in (None, em):
            want = ref.reduce(ref.PROD, off, content, obj_mask=om, evt_mask=evm)
            got = H.reduce(H.PROD, dev(off), dcontent, obj_mask=None if om is None or om.size == 0 else dev(om),
                           evt_mask=None if evm is None else dev(evm)).cpu().numpy()
            assert_same_f32(got, want, f"prod n={n_events}")
    if n_events and content.size:
        c16 = content.astype(np.float16)
        assert_same_f32(H.reduce(H.PROD, dev(off), dev(c16)).cpu().numpy(),
                        ref.reduce(ref.PROD, off, c16), "prod f16")


def test_reduce_prod_order_and_big_events():
    """Order-sensitive products (rounding differs left to right vs any other
    order) and events beyond the staged tile (walked from HBM)."""
    say("reduce PROD order")
    sizes = np.array([3, 0, 1, 700, 2, 1300, 5], np.int64)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    rng = np.random.default_rng(9)
    c = rng.uniform(0.999, 1.001, int(off[-1])).astype(np.float32)
    c[:3] = [np.float32(1 + 2 ** -23), np.float32(1 + 2 ** -23), np.float32(1 - 2 ** -24)]
    want = ref.reduce(ref.PROD, off, c)
    got = H.reduce(H.PROD, dev(off), dev(c)).cpu().numpy()
    assert_same_f32(got, want, "prod order")


@pytest.mark.parametrize("n,nbins", [(0, 10), (100003, 100), (100003, 2500), (5001, 21)])
def test_hist_fill_w2(n, nbins):
    say(f"hist_fill_w2 n={n} nbins={nbins}")
    import torch
    rng = np.random.default_rng(n + nbins)
    x = rng.uniform(-5, 105, n).astype(np.float32)
    if n > 10:
        x[:3] = [np.nan, 100.0, 0.0]
    w = rng.normal(1.0, 0.1, n).astype(np.float32)
    m = (rng.uniform(size=n) < 0.6).astype(np.uint8)
    edges = datagen.uniform_edges(nbins, 0.0, 100.0)
    sumw, sumw2, counts = ref.hist_fill_w2(x, edges, w=w, evt_mask=m)
    s = torch.zeros(nbins + 2, dtype=torch.float64, device="cuda")
    s2 = torch.zeros(nbins + 2, dtype=torch.float64, device="cuda")
    c = torch.zeros(nbins + 2, dtype=torch.int64, device="cuda")
    for _ in range(2):  # accumulates
        H.hist_fill(dev(x), dev(edges), s, c, w=dev(w), evt_mask=dev(m), sumw2=s2)
    assert np.array_equal(c.cpu().numpy().astype(np.uint64), 2 * counts)
    for got, want in ((s, sumw), (s2, sumw2)):
        g = got.cpu().numpy()
        assert np.all(np.abs(g - 2 * want) <= RTOL * np.abs(2 * want))
    # without weights: every squared weight is 1
    s2.zero_()
    s.zero_()
    c.zero_()
    H.hist_fill(dev(x), dev(edges), s, c, sumw2=s2)
    assert np.array_equal(s2.cpu().numpy(), s.cpu().numpy())
