"""Pins of the oracle's positional kernels (Sec. III get_in_offsets,
set_in_offsets, select_opposite_sign_muons), compaction and top-quark
triplet search (Sec. IV), against definitions written out independently:
plain Python loops over tiny seeded events, numpy boolean indexing,
itertools over triplets in float32 scalar arithmetic, float64 numpy
four-momenta, and hand-built events whose answers follow by hand.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import ref

F = np.float32


def jagged(seed, n_events, mean=3.0, cap=9):
    rng = np.random.default_rng(seed)
    counts = np.minimum(rng.poisson(mean, n_events), cap)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    return rng, off, int(off[-1])


# ---------------------------------------------------------------- get / set

def brute_nth(off, mask, e, n):
    sel = [i for i in range(off[e], off[e + 1]) if mask is None or mask[i]]
    return sel[n] if 0 <= n < len(sel) else -1


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_get_in_offsets_brute_force(seed):
    rng, off, m = jagged(seed, 300)
    c = rng.normal(50, 20, m).astype(F)
    mask = (rng.uniform(size=m) < 0.6).astype(np.uint8)
    emask = (rng.uniform(size=300) < 0.8).astype(np.uint8)
    idx = rng.integers(-1, 5, 300).astype(np.int32)
    for om in (None, mask):
        for em in (None, emask):
            for n, ix in ((0, None), (2, None), (-1, None), (0, idx)):
                got, gi = ref.get_in_offsets(off, c, n=n, idx=ix, obj_mask=om, evt_mask=em, fill=-7.5)
                for e in range(300):
                    k = int(ix[e]) if ix is not None else n
                    i = -1 if (em is not None and not em[e]) else brute_nth(off, om, e, k)
                    assert gi[e] == (i - off[e] if i >= 0 else -1)
                    assert got[e] == (c[i] if i >= 0 else F(-7.5))


def test_get_in_offsets_float16_and_hand_event():
    off = np.array([0, 3, 3, 5], np.int64)
    c = np.array([10, 20, 30, 40, 50], np.float16)
    mask = np.array([0, 1, 1, 1, 0], np.uint8)
    got, gi = ref.get_in_offsets(off, c, n=1, obj_mask=mask, fill=0.0)
    assert got.tolist() == [30.0, 0.0, 0.0] and gi.tolist() == [2, -1, -1]
    got, gi = ref.get_in_offsets(off, c, n=0, obj_mask=mask)
    assert got.tolist() == [20.0, 0.0, 40.0] and gi.tolist() == [1, -1, 0]


@pytest.mark.parametrize("seed", [3, 4])
def test_set_in_offsets_brute_force(seed):
    rng, off, m = jagged(seed, 200)
    mask = (rng.uniform(size=m) < 0.5).astype(np.uint8)
    emask = (rng.uniform(size=200) < 0.7).astype(np.uint8)
    c = rng.normal(0, 1, m).astype(F)
    got = ref.set_in_offsets(off, c, 9.0, n=1, obj_mask=mask, evt_mask=emask)
    want = c.copy()
    for e in range(200):
        i = brute_nth(off, mask, e, 1) if emask[e] else -1
        if i >= 0:
            want[i] = 9.0
    assert np.array_equal(got.view(np.uint32), want.view(np.uint32))
    # a mask of the first two selected objects of every event, built with two calls
    z = np.zeros(m, np.uint8)
    z = ref.set_in_offsets(off, z, 1.0, n=0, obj_mask=mask)
    z = ref.set_in_offsets(off, z, 1.0, n=1, obj_mask=mask)
    for e in range(200):
        sel = [i for i in range(off[e], off[e + 1]) if mask[i]]
        assert [i for i in range(off[e], off[e + 1]) if z[i]] == sel[:2]
    # value 0 clears
    assert not np.any(ref.set_in_offsets(off, np.ones(m, np.uint8), 0.0, n=0)[off[:-1][np.diff(off) > 0]])


# ---------------------------------------------------------------- opposite sign

def brute_opposite(off, pt, q, mask):
    out = np.zeros(len(pt), np.uint8)
    for e in range(len(off) - 1):
        sel = [i for i in range(off[e], off[e + 1]) if mask is None or mask[i]]
        # pT order: numbers before NaN, larger first, then lower index
        order = sorted(sel, key=lambda i: (math.isnan(pt[i]), -pt[i] if not math.isnan(pt[i]) else 0.0, i))
        done = False
        for p in range(len(order)):
            for r in range(p + 1, len(order)):
                a, b = q[order[p]], q[order[r]]
                if (a > 0 > b) or (a < 0 < b):
                    out[order[p]] = out[order[r]] = 1
                    done = True
                    break
            if done:
                break
    return out


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_opposite_sign_brute_force(seed):
    rng, off, m = jagged(seed, 400, mean=2.5, cap=8)
    pt = np.round(rng.exponential(30, m) + 20).astype(F)  # rounded: equal pt occurs
    pt[rng.integers(0, m, m // 40)] = np.nan
    q = rng.choice(np.array([-1, 1, 0, 2, -2], np.int32), m, p=[0.45, 0.45, 0.04, 0.03, 0.03])
    mask = (rng.uniform(size=m) < 0.8).astype(np.uint8)
    for om in (None, mask):
        assert np.array_equal(ref.select_opposite_sign(off, pt, q, om), brute_opposite(off, pt, q, om))


def test_opposite_sign_hand_events():
    # event 0: pt 50(+), 40(+), 30(-) -> the leading muon and the 30 GeV one
    # event 1: all positive -> none; event 2: stored out of pT order
    # event 3: equal pt -> lower index first; event 4: the leading object has
    # charge 0, so the pair starts at the second
    off = np.array([0, 3, 5, 8, 11, 14], np.int64)
    pt = np.array([50, 40, 30, 60, 70, 25, 80, 45, 30, 30, 30, 90, 50, 40], F)
    q = np.array([1, 1, -1, 1, 1, -1, 1, -1, 1, 1, -1, 0, 1, -1], np.int32)
    got = ref.select_opposite_sign(off, pt, q)
    assert got.tolist() == [1, 0, 1, 0, 0, 0, 1, 1, 1, 0, 1, 0, 1, 1]


# ---------------------------------------------------------------- compaction

@pytest.mark.parametrize("dtype", [np.float32, np.float16, np.int32, np.uint8])
def test_compact_is_boolean_indexing(dtype):
    rng, off, m = jagged(8, 500)
    c = (rng.normal(0, 50, m)).astype(dtype)
    mask = (rng.uniform(size=m) < 0.4).astype(np.uint8)
    got = ref.compact(off, c, mask)
    want = c[mask.astype(bool)]
    assert got.dtype == want.dtype and np.array_equal(got.view(np.uint8), want.view(np.uint8))
    assert np.array_equal(ref.compact(off, c), c)
    # its layout is that of the counts' prefix offsets
    cnt, offo = ref.reduce(ref.COUNT, off, obj_mask=mask, want_offsets=True)
    assert offo[-1] == len(got)
    for e in range(0, 500, 37):
        sel = [i for i in range(off[e], off[e + 1]) if mask[i]]
        assert np.array_equal(got[offo[e]:offo[e + 1]].view(np.uint8), c[sel].view(np.uint8))


# ---------------------------------------------------------------- four-momenta

def test_p4_against_float64_numpy():
    rng = np.random.default_rng(9)
    n = 5000
    pt = (20 + rng.exponential(30, n)).astype(F)
    eta = np.clip(rng.normal(0, 1.5, n), -4.7, 4.7).astype(F)
    phi = rng.uniform(-np.pi, np.pi, n).astype(F)
    mass = rng.uniform(0, 20, n).astype(F)
    px, py, pz, en = ref.p4(pt, eta, phi, mass)
    p, h, f, m = (a.astype(np.float64) for a in (pt, eta, phi, mass))
    x, y, z = p * np.cos(f), p * np.sin(f), p * np.sinh(h)
    e = np.sqrt(x * x + y * y + z * z + m * m)
    for got, want in ((px, x), (py, y), (pz, z), (en, e)):
        # both round a float64 value once: within one float32 ulp
        assert np.all(np.abs(got.astype(np.float64) - want) <= np.spacing(np.abs(want).astype(F)).astype(np.float64))
    # invariant: E^2 - |p|^2 = m^2, up to the float32 rounding of each
    # component (relative 2^-24 each, so a few 2^-24 of E^2 in the difference)
    e64 = en.astype(np.float64)
    p2 = px.astype(np.float64) ** 2 + py.astype(np.float64) ** 2 + pz.astype(np.float64) ** 2
    assert np.all(np.abs((e64 * e64 - p2) - m * m) <= 8 * 2.0 ** -24 * e64 * e64)


def test_p4_float16_widening():
    pt = np.array([30.0, 45.5], np.float16)
    z = np.zeros(2, np.float16)
    px, py, pz, en = ref.p4(pt, z, z, z)
    assert px.tolist() == [30.0, 45.5] and py.tolist() == [0.0, 0.0] and en.tolist() == [30.0, 45.5]


# ---------------------------------------------------------------- triplets

def brute_triplet(off, X, Y, Z, E, mask, target):
    nev = len(off) - 1
    mass = np.full(nev, np.nan, F)
    idx = np.full((nev, 3), -1, np.int32)
    t = F(target)
    for e in range(nev):
        sel = [i for i in range(off[e], off[e + 1]) if mask is None or mask[i]]
        best = F(np.inf)
        for i, j, k in itertools.combinations(sel, 3):
            sx = (X[i] + X[j]) + X[k]
            sy = (Y[i] + Y[j]) + Y[k]
            sz = (Z[i] + Z[j]) + Z[k]
            se = (E[i] + E[j]) + E[k]
            m2 = ((se * se - sx * sx) - sy * sy) - sz * sz
            mm = F(0) if m2 < 0 else np.sqrt(m2)
            d = abs(mm - t)
            if d < best:
                best, mass[e] = d, mm
                idx[e] = [i - off[e], j - off[e], k - off[e]]
    return mass, idx


@pytest.mark.parametrize("seed", [10, 11])
def test_best_triplet_brute_force(seed):
    rng, off, m = jagged(seed, 250, mean=5.0, cap=12)
    pt = (20 + rng.exponential(30, m)).astype(F)
    eta = np.clip(rng.normal(0, 1.5, m), -4.7, 4.7).astype(F)
    phi = rng.uniform(-np.pi, np.pi, m).astype(F)
    mass = rng.uniform(0, 20, m).astype(F)
    X, Y, Z, E = ref.p4(pt, eta, phi, mass)
    X[rng.integers(0, m, 5)] = np.nan
    mask = (rng.uniform(size=m) < 0.7).astype(np.uint8)
    with np.errstate(invalid="ignore"):
        for om in (None, mask):
            gm, gi = ref.best_triplet(off, X, Y, Z, E, om, 172.0)
            wm, wi = brute_triplet(off, X, Y, Z, E, om, 172.0)
            assert np.array_equal(gi, wi)
            assert np.array_equal(np.isnan(gm), np.isnan(wm))
            ok = ~np.isnan(wm)
            assert np.array_equal(gm[ok].view(np.uint32), wm[ok].view(np.uint32))


def test_best_triplet_hand_events():
    # event 0 (four objects): two back-to-back massless 86 GeV jets (0, 1), a
    # 10 GeV mass at rest (2) and a massless 20 GeV jet along z (3).  By hand:
    # (0,1,2): E = 182, p = 0 -> M = 182; (0,1,3): E = 192, p = 20 ->
    # M = sqrt(192^2 - 20^2) = 190.96; (0,2,3) and (1,2,3): E = 116,
    # |p|^2 = 86^2 + 20^2 -> M = 75.2.  Closest to 172: (0,1,2).
    # event 1: two objects, no triplet.
    X = np.array([86, -86, 0, 0, 1, 2], F)
    Y = np.zeros(6, F)
    Z = np.array([0, 0, 0, 20, 0, 0], F)
    E = np.array([86, 86, 10, 20, 1, 2], F)
    off = np.array([0, 4, 6], np.int64)
    m, idx = ref.best_triplet(off, X, Y, Z, E, None, 172.0)
    assert idx[0].tolist() == [0, 1, 2] and m[0] == F(182.0)
    assert np.isnan(m[1]) and idx[1].tolist() == [-1, -1, -1]
    # ties: two identical triplets, the first wins
    X2 = np.array([50, -50, 0, 0], F)
    E2 = np.array([50, 50, 72, 72], F)
    m2, i2 = ref.best_triplet(np.array([0, 4], np.int64), X2, np.zeros(4, F), np.zeros(4, F), E2, None, 172.0)
    assert i2[0].tolist() == [0, 1, 2] and m2[0] == F(172.0)
