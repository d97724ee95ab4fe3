"""GPU parity of the positional kernels, compaction and the top-quark
triplet search against the CPU oracle.

hepk_get_in_offsets / hepk_set_in_offsets / hepk_select_opposite_sign /
hepk_compact / hepk_best_triplet must equal the oracle bit for bit
(indices, masks, moved elements, float32 masses); hepk_p4 uses the device's
float32 cos/sin/sinh and is compared with the oracle's float64 values within
a few float32 ulp.  Inputs: the seeded analysis events (jets and muons, with
a synthetic charge column), non-finite values, equal pt, masked and empty
events, float16 content, and events dense enough to exceed the kernels' LDS
staging.
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


def dev(a):
    import torch
    a = np.ascontiguousarray(a)
    if a.size == 0:  # a valid pointer for a column of no objects
        a = np.zeros(1, a.dtype)
    return torch.from_numpy(a).to("cuda")


def u32(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def jets_of(n, seed, dtype="f32"):
    ds = datagen.make_dataset(seed, n, content_dtype=dtype)
    return ds, ds.jets


def dense_jets(seed):
    """Events with 12 to 20 objects (tiles beyond the staging capacity)."""
    rng = np.random.default_rng(seed)
    counts = rng.integers(12, 21, 300)
    counts[:3] = [0, 1, 2]
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    m = int(off[-1])
    cols = {"pt": (20 + rng.exponential(30, m)).astype(np.float32),
            "eta": np.clip(rng.normal(0, 1.5, m), -4.7, 4.7).astype(np.float32),
            "phi": rng.uniform(-np.pi, np.pi, m).astype(np.float32),
            "mass": rng.uniform(0, 20, m).astype(np.float32)}
    return off, cols


@pytest.mark.parametrize("n", [0, 1, 1000, 100003])
def test_get_and_set_in_offsets(n):
    say(f"get/set n={n}")
    ds, j = jets_of(n, 70)
    off, pt = j.offsets, j.cols["pt"]
    rng = np.random.default_rng(n)
    m = j.n_objects
    mask = ((pt > 30) & (np.abs(j.cols["eta"]) < 2.5)).astype(np.uint8)
    em = (rng.uniform(size=n) < 0.8).astype(np.uint8)
    idx = rng.integers(-1, 6, n).astype(np.int32)
    for om in (None, mask):
        for evm in (None, em):
            for k, ix in ((0, None), (1, None), (3, None), (-1, None), (0, idx)):
                wv, wi = ref.get_in_offsets(off, pt, n=k, idx=ix, obj_mask=om, evt_mask=evm, fill=-1.0)
                gv, gi = H.get_in_offsets(dev(off), dev(pt), n=k, idx=None if ix is None else dev(ix),
                                          obj_mask=None if om is None else dev(om),
                                          evt_mask=None if evm is None else dev(evm), fill=-1.0)
                assert np.array_equal(u32(gv.cpu().numpy()[:n]), u32(wv)), f"get n={k}"
                assert np.array_equal(gi.cpu().numpy()[:n], wi), f"get index n={k}"
    if n:
        p16 = pt.astype(np.float16)
        wv, wi = ref.get_in_offsets(off, p16, n=2, obj_mask=mask)
        gv, gi = H.get_in_offsets(dev(off), dev(p16), n=2, obj_mask=dev(mask))
        assert np.array_equal(u32(gv.cpu().numpy()), u32(wv)) and np.array_equal(gi.cpu().numpy(), wi)
    # set: a mask of the first two selected jets, and a float column
    z = np.zeros(m, np.uint8)
    want = ref.set_in_offsets(off, ref.set_in_offsets(off, z, 1.0, n=0, obj_mask=mask), 1.0, n=1, obj_mask=mask)
    gz = dev(z)
    H.set_in_offsets(dev(off), gz, 1.0, n=0, obj_mask=dev(mask))
    H.set_in_offsets(dev(off), gz, 1.0, n=1, obj_mask=dev(mask))
    assert np.array_equal(gz.cpu().numpy()[:m], want)
    want = ref.set_in_offsets(off, pt, -3.5, idx=idx, evt_mask=em)
    gp = dev(pt.copy())
    H.set_in_offsets(dev(off), gp, -3.5, idx=dev(idx), evt_mask=dev(em))
    assert np.array_equal(u32(gp.cpu().numpy()[:m]), u32(want))


@pytest.mark.parametrize("n", [0, 5, 20000, 100003])
def test_opposite_sign(n):
    say(f"opposite sign n={n}")
    ds = datagen.make_dataset(71, n)
    mu = ds.muons
    q = datagen.muon_charges(ds, 71)
    pt = np.round(mu.cols["pt"]).astype(np.float32)  # equal pt within events occurs
    rng = np.random.default_rng(n + 1)
    if mu.n_objects > 50:
        pt[rng.integers(0, mu.n_objects, mu.n_objects // 50)] = np.nan
        q[rng.integers(0, mu.n_objects, mu.n_objects // 50)] = 0
    msel = ((mu.cols["pt"] > 20) & (np.abs(mu.cols["eta"]) < 2.4) & (mu.cols["iso"] < 0.15)).astype(np.uint8)
    for om in (None, msel):
        want = ref.select_opposite_sign(mu.offsets, pt, q, om)
        got = H.select_opposite_sign(dev(mu.offsets), dev(pt), dev(q), None if om is None else dev(om))
        assert np.array_equal(got.cpu().numpy()[:mu.n_objects], want)
    if n:
        p16 = pt.astype(np.float16)
        want = ref.select_opposite_sign(mu.offsets, p16, q, msel)
        got = H.select_opposite_sign(dev(mu.offsets), dev(p16), dev(q), dev(msel))
        assert np.array_equal(got.cpu().numpy()[:mu.n_objects], want)


def test_opposite_sign_dense_events():
    say("opposite sign dense")
    off, cols = dense_jets(72)
    rng = np.random.default_rng(72)
    q = np.where(rng.uniform(size=int(off[-1])) < 0.9, 1, -1).astype(np.int32)
    want = ref.select_opposite_sign(off, cols["pt"], q)
    assert np.array_equal(H.select_opposite_sign(dev(off), dev(cols["pt"]), dev(q)).cpu().numpy(), want)


@pytest.mark.parametrize("dtype", [np.float32, np.float16, np.int32, np.uint8])
@pytest.mark.parametrize("n", [0, 1, 777, 100003])
def test_compact(n, dtype):
    say(f"compact n={n} {np.dtype(dtype).name}")
    ds, j = jets_of(n, 73)
    off = j.offsets
    m = j.n_objects
    rng = np.random.default_rng(n)
    c = rng.normal(0, 1000, m).astype(dtype)
    mask = ((j.cols["pt"] > 30) & (np.abs(j.cols["eta"]) < 2.5)).astype(np.uint8)
    for om in (None, mask):
        want = ref.compact(off, c, om)
        cnt, offo = H.reduce(H.COUNT, dev(off), obj_mask=None if om is None else dev(om), want_offsets=True)
        n_out = int(offo[-1].item()) if n else 0
        assert n_out == len(want)
        got = H.compact(dev(off), dev(c), offo, n_out, obj_mask=None if om is None else dev(om))
        assert np.array_equal(got.cpu().numpy().view(np.uint8), want.view(np.uint8))
    if n > 100:
        # a smaller output bound: nothing is written beyond it
        import torch
        cnt, offo = H.reduce(H.COUNT, dev(off), obj_mask=dev(mask), want_offsets=True)
        out = torch.full((int(offo[-1].item()),), 0x5A, dtype=torch.uint8, device="cuda")
        if dtype == np.uint8:
            H.compact(dev(off), dev(c), offo, 10, obj_mask=dev(mask), out=out)
            got = out.cpu().numpy()
            assert np.array_equal(got[:10], ref.compact(off, c, mask)[:10]) and np.all(got[10:] == 0x5A)


@pytest.mark.parametrize("dtype", [np.float32, np.float16, np.uint8])
def test_compact_dense_tiles(dtype):
    """Tiles of more objects than the kernel reads in one batch (events of
    12 to 20 objects), and tiles on either side of that bound."""
    say(f"compact dense {np.dtype(dtype).name}")
    off, cols = dense_jets(77)
    counts = np.diff(off)
    # events of 8 objects: 512 per tile, exactly the batch; then 9: 576
    counts = np.concatenate([counts, np.full(64, 8), np.full(64, 9), counts[:50]])
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    m = int(off[-1])
    rng = np.random.default_rng(77)
    c = rng.normal(0, 1000, m).astype(dtype)
    mask = (rng.uniform(size=m) < 0.7).astype(np.uint8)
    for om in (None, mask):
        want = ref.compact(off, c, om)
        cnt, offo = H.reduce(H.COUNT, dev(off), obj_mask=None if om is None else dev(om), want_offsets=True)
        n_out = int(offo[-1].item())
        assert n_out == len(want)
        got = H.compact(dev(off), dev(c), offo, n_out, obj_mask=None if om is None else dev(om))
        assert np.array_equal(got.cpu().numpy().view(np.uint8), want.view(np.uint8))


def test_p4_within_float32_ulps():
    say("p4")
    ds, j = jets_of(100003, 74)
    c = j.cols
    want = ref.p4(c["pt"], c["eta"], c["phi"], c["mass"])
    got = [a.cpu().numpy() for a in H.p4(dev(c["pt"]), dev(c["eta"]), dev(c["phi"]), dev(c["mass"]))]
    ulp = 2.0 ** -24
    pt = c["pt"].astype(np.float64)
    # px, py: cos/sin to a few ulp, times pt; pz: sinh to a few ulp; E: sum of squares and sqrt
    scale = (pt, pt, np.abs(want[2].astype(np.float64)) + pt, want[3].astype(np.float64))
    for g, w, s, name in zip(got, want, scale, ("px", "py", "pz", "E")):
        err = np.abs(g.astype(np.float64) - w.astype(np.float64))
        assert np.all(err <= 16 * ulp * s), f"{name}: max err / scale {np.max(err / s) / ulp:.1f} ulp"


def test_p4_vector_and_row_kernels_agree():
    """Columns offset by one object (not 16-byte aligned: one object per
    thread) and the same values in fresh allocations (four objects per thread,
    the n % 4 last ones one per thread) give the same bits."""
    import torch
    say("p4 vector and row kernels")
    ds, j = jets_of(50001, 75)
    c = j.cols
    n = c["pt"].size - (1 if c["pt"].size % 4 == 0 else 0)
    cols = [dev(np.concatenate([[0.0], c[k][:n]]).astype(np.float32)) for k in ("pt", "eta", "phi", "mass")]
    rows = H.p4(*[x[1:] for x in cols])
    vec = H.p4(*[x[1:].clone() for x in cols])
    assert n % 4 != 0
    for u, v, name in zip(rows, vec, ("px", "py", "pz", "E")):
        assert torch.equal(u.view(torch.int32), v.view(torch.int32)), name


@pytest.mark.parametrize("source", ["analysis", "dense"])
def test_best_triplet_bit_exact(source):
    say(f"best triplet {source}")
    if source == "analysis":
        ds, j = jets_of(100003, 75)
        off, c = j.offsets, j.cols
        mask = ((c["pt"] > 30) & (np.abs(c["eta"]) < 2.5)).astype(np.uint8)
    else:
        off, c = dense_jets(76)
        mask = (np.random.default_rng(76).uniform(size=int(off[-1])) < 0.8).astype(np.uint8)
    X, Y, Z, E = ref.p4(c["pt"], c["eta"], c["phi"], c["mass"])
    if len(X) > 100:
        X[::97] = np.nan  # triplets with a NaN mass are never chosen
    for om in (None, mask):
        wm, wi = ref.best_triplet(off, X, Y, Z, E, om, 172.0)
        gm, gi = H.best_triplet(dev(off), dev(X), dev(Y), dev(Z), dev(E), None if om is None else dev(om), 172.0)
        gm, gi = gm.cpu().numpy(), gi.cpu().numpy()
        assert np.array_equal(gi, wi)
        assert np.array_equal(np.isnan(gm), np.isnan(wm))
        ok = ~np.isnan(wm)
        assert np.array_equal(u32(gm[ok]), u32(wm[ok]))


def test_best_triplet_chain_from_device_p4():
    """p4 then the triplet search, all on the device, against the oracle's
    chain: masses agree to float32 rounding, and a different triplet is
    chosen only where two candidates are that close to the target."""
    say("triplet chain")
    ds, j = jets_of(50000, 77)
    c = j.cols
    off = j.offsets
    mask = ((c["pt"] > 30) & (np.abs(c["eta"]) < 2.5)).astype(np.uint8)
    wm, wi = ref.best_triplet(off, *ref.p4(c["pt"], c["eta"], c["phi"], c["mass"]), mask, 172.0)
    gp = H.p4(dev(c["pt"]), dev(c["eta"]), dev(c["phi"]), dev(c["mass"]))
    gm, gi = H.best_triplet(dev(off), *gp, dev(mask), 172.0)
    gm, gi = gm.cpu().numpy(), gi.cpu().numpy()
    assert np.array_equal(np.isnan(gm), np.isnan(wm))
    ok = ~np.isnan(wm)
    same = np.all(gi == wi, axis=1) & ok
    # the same triplet: its mass to the rounding of the device's four-momenta
    assert np.all(np.abs(gm[same] - wm[same]) <= 1e-3 * np.maximum(wm[same], 1.0))
    # another triplet: only where the two are equally close to the target
    other = ok & ~same
    assert np.all(np.abs(np.abs(gm[other] - 172) - np.abs(wm[other] - 172)) <= 1e-3 * np.maximum(wm[other], 1.0))
    assert np.mean(same[ok]) > 0.999
