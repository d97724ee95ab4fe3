"""Python access to the CPU oracle (hepkref.c) on numpy arrays.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The GPU library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import List, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hepkref.c")
LIB = os.environ.get("HEPKREF_LIB") or os.path.join(HERE, "libhepkref.so")

# float32 cut arithmetic rounded operation by operation: no contraction into
# fused multiply-adds and no fast-math reassociation.
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
          "-Wall", "-Wextra", "-Wno-unused-parameter"]

F32, F16, I32, U8 = 0, 1, 2, 3
GT, GE, LT, LE, ABS_LT, ABS_LE = range(6)
COUNT, SUM, MAX, MIN, ARGMAX, ARGMIN, PROD = range(7)


def build(force: bool = False, extra_flags: Sequence[str] = ()) -> str:
    """Compile libhepkref.so with gcc (also the "does it build" step)."""
    if os.environ.get("HEPKREF_LIB"):
        return LIB
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(SRC), os.path.getmtime(os.path.join(HERE, "hepkref.h"))):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, *extra_flags, "-shared", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Cut(C.Structure):
    _fields_ = [("col", C.c_void_p), ("dtype", C.c_int32), ("op", C.c_int32),
                ("thr", C.c_float), ("ithr", C.c_int32)]


class Coll(C.Structure):
    _fields_ = [("off", C.c_void_p), ("pt", C.c_void_p), ("eta", C.c_void_p),
                ("phi", C.c_void_p), ("extra", C.c_void_p)]


class DatasetS(C.Structure):
    _fields_ = [("n_events", C.c_int64), ("dtype", C.c_int32),
                ("jets", Coll), ("muons", Coll), ("electrons", Coll),
                ("weights", C.c_void_p), ("npu", C.c_void_p)]


class QueryS(C.Structure):
    _fields_ = [("mu_pt", C.c_float), ("mu_abseta", C.c_float), ("mu_iso", C.c_float),
                ("el_pt", C.c_float), ("el_abseta", C.c_float),
                ("jet_pt", C.c_float), ("jet_abseta", C.c_float),
                ("dr", C.c_float), ("btag", C.c_float),
                ("min_mu", C.c_int32), ("min_jet", C.c_int32), ("min_b", C.c_int32),
                ("n_scale", C.c_int32), ("scales", C.c_void_p),
                ("edges", C.c_void_p * 3), ("nbins", C.c_int32 * 3),
                ("pu_edges", C.c_void_p), ("pu_contents", C.c_void_p), ("pu_nbins", C.c_int32),
                ("sf_edges", C.c_void_p), ("sf_contents", C.c_void_p), ("sf_nbins", C.c_int32),
                ("jes_mode", C.c_int32), ("jes_eta_edges", C.c_void_p), ("jes_pt_edges", C.c_void_p),
                ("jes_delta", C.c_void_p), ("jes_n_eta", C.c_int32), ("jes_n_pt", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        _lib.hepkref_half_to_float.restype = C.c_float
        _lib.hepkref_half_to_float.argtypes = [C.c_uint16]
        _lib.hepkref_select.argtypes = [C.POINTER(Cut), C.c_int32, C.c_int64, C.c_void_p, C.c_void_p]
        _lib.hepkref_reduce.argtypes = [C.c_int32, C.c_void_p, C.c_int64, C.c_void_p, C.c_int32,
                                        C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.hepkref_match_dr.argtypes = [C.c_void_p] * 4 + [C.c_void_p] * 4 + [
            C.c_int32, C.c_int64, C.c_float, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.hepkref_hist_fill.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                           C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        _lib.hepkref_hist_fill_w2.argtypes = [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int64,
                                              C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
        _lib.hepkref_get_bin_contents.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32,
                                                  C.c_void_p, C.c_void_p]
        _lib.hepkref_interp.argtypes = [C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32,
                                        C.c_void_p, C.c_void_p]
        _lib.hepkref_jes_delta.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_int64, C.c_void_p, C.c_int32,
                                           C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]
        _lib.hepkref_get_in_offsets.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_int32, C.c_float, C.c_void_p,
                                                C.c_void_p]
        _lib.hepkref_set_in_offsets.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                                C.c_void_p, C.c_void_p, C.c_int32, C.c_float]
        _lib.hepkref_select_opposite_sign.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p,
                                                      C.c_void_p, C.c_void_p]
        _lib.hepkref_compact.argtypes = [C.c_void_p, C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p,
                                         C.c_void_p]
        _lib.hepkref_p4.argtypes = [C.c_void_p] * 4 + [C.c_int32, C.c_int64] + [C.c_void_p] * 4
        _lib.hepkref_best_triplet.argtypes = [C.c_void_p, C.c_int64] + [C.c_void_p] * 5 + [
            C.c_float, C.c_void_p, C.c_void_p]
        _lib.hepkref_pipeline.argtypes = [C.POINTER(DatasetS), C.POINTER(QueryS), C.c_int32,
                                          C.c_void_p, C.c_void_p, C.c_void_p]
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _dt(a: np.ndarray) -> int:
    return {np.dtype(np.float32): F32, np.dtype(np.float16): F16,
            np.dtype(np.int32): I32}[a.dtype]


def _check(rc):
    if rc != 0:
        raise ValueError(f"oracle returned {rc}")


def half_to_float(h: int) -> float:
    return lib().hepkref_half_to_float(h)


def select(cuts, n: int, mask_in=None) -> np.ndarray:
    """cuts: list of (column array, op, threshold)."""
    arr = (Cut * max(1, len(cuts)))()
    keep = []
    for i, (col, op, thr) in enumerate(cuts):
        col = np.ascontiguousarray(col)
        keep.append(col)
        if col.dtype == np.int32:
            arr[i] = Cut(col.ctypes.data, I32, op, 0.0, int(thr))
        else:
            arr[i] = Cut(col.ctypes.data, _dt(col), op, float(thr), 0)
    out = np.empty(n, np.uint8)
    _check(lib().hepkref_select(arr, len(cuts), n, _p(mask_in), out.ctypes.data))
    return out


def reduce(op: int, offsets: np.ndarray, content=None, obj_mask=None, evt_mask=None,
           want_arg: bool = False, want_offsets: bool = False):
    n = len(offsets) - 1
    if content is not None:
        content = np.ascontiguousarray(content)
    if op in (COUNT, ARGMAX, ARGMIN):
        out = np.empty(n, np.int32)
    else:
        out = np.empty(n, np.float32)
    arg = np.empty(n, np.int32) if want_arg else None
    offo = np.empty(n + 1, np.int64) if want_offsets else None
    dt = _dt(content) if content is not None else F32
    _check(lib().hepkref_reduce(op, offsets.ctypes.data, n, _p(content), dt,
                                _p(obj_mask), _p(evt_mask), out.ctypes.data,
                                _p(arg), _p(offo)))
    res = [out]
    if want_arg:
        res.append(arg)
    if want_offsets:
        res.append(offo)
    return res[0] if len(res) == 1 else tuple(res)


def match_dr(off_a, eta_a, phi_a, off_b, eta_b, phi_b, dr: float,
             mask_a=None, mask_b=None):
    """Returns (min_dr2 float32[Ma], idx int32[Ma], clean uint8[Ma])."""
    ma = int(off_a[-1])
    md = np.empty(ma, np.float32)
    ix = np.empty(ma, np.int32)
    cl = np.empty(ma, np.uint8)
    _check(lib().hepkref_match_dr(off_a.ctypes.data, eta_a.ctypes.data, phi_a.ctypes.data,
                                  _p(mask_a), off_b.ctypes.data, eta_b.ctypes.data,
                                  phi_b.ctypes.data, _p(mask_b), _dt(eta_a), len(off_a) - 1,
                                  dr, md.ctypes.data, ix.ctypes.data, cl.ctypes.data))
    return md, ix, cl


def hist_fill(x, edges, w=None, evt_mask=None, sumw=None, counts=None):
    nb = len(edges) - 1
    if sumw is None:
        sumw = np.zeros(nb + 2, np.float64)
    if counts is None:
        counts = np.zeros(nb + 2, np.uint64)
    edges = np.ascontiguousarray(edges, np.float32)
    _check(lib().hepkref_hist_fill(x.ctypes.data, _dt(x), _p(w), _p(evt_mask), len(x),
                                   edges.ctypes.data, nb, sumw.ctypes.data, counts.ctypes.data))
    return sumw, counts


def hist_fill_w2(x, edges, w=None, evt_mask=None):
    """(sumw, sumw2, counts) of a fresh histogram."""
    nb = len(edges) - 1
    sumw, sumw2 = np.zeros(nb + 2, np.float64), np.zeros(nb + 2, np.float64)
    counts = np.zeros(nb + 2, np.uint64)
    edges = np.ascontiguousarray(edges, np.float32)
    _check(lib().hepkref_hist_fill_w2(x.ctypes.data, _dt(x), _p(w), _p(evt_mask), len(x), edges.ctypes.data,
                                      nb, sumw.ctypes.data, sumw2.ctypes.data, counts.ctypes.data))
    return sumw, sumw2, counts


def get_bin_contents(x, edges, contents) -> np.ndarray:
    """Lookup-histogram content of each element (contents: nbins+2 slots)."""
    x = np.ascontiguousarray(x)
    edges = np.ascontiguousarray(edges, np.float32)
    contents = np.ascontiguousarray(contents, np.float32)
    out = np.empty(len(x), np.float32)
    _check(lib().hepkref_get_bin_contents(x.ctypes.data, _dt(x), len(x), edges.ctypes.data, len(edges) - 1,
                                          contents.ctypes.data, out.ctypes.data))
    return out


def interp(x, edges, contents) -> np.ndarray:
    """Linear interpolation between bin centres (contents: nbins+2 slots)."""
    x = np.ascontiguousarray(x)
    edges = np.ascontiguousarray(edges, np.float32)
    contents = np.ascontiguousarray(contents, np.float32)
    out = np.empty(len(x), np.float32)
    _check(lib().hepkref_interp(x.ctypes.data, _dt(x), len(x), edges.ctypes.data, len(edges) - 1,
                                contents.ctypes.data, out.ctypes.data))
    return out


def jes_delta(pt, eta, eta_edges, pt_edges, delta) -> np.ndarray:
    """Per-object shift from a (|eta| row, interpolated pt) table."""
    pt, eta = np.ascontiguousarray(pt), np.ascontiguousarray(eta)
    ee = np.ascontiguousarray(eta_edges, np.float32)
    pe = np.ascontiguousarray(pt_edges, np.float32)
    d = np.ascontiguousarray(delta, np.float32)
    out = np.empty(len(pt), np.float32)
    _check(lib().hepkref_jes_delta(pt.ctypes.data, eta.ctypes.data, _dt(pt), len(pt), ee.ctypes.data,
                                   len(ee) - 1, pe.ctypes.data, len(pe) - 1, d.ctypes.data, out.ctypes.data))
    return out


def get_in_offsets(offsets, content, n: int = 0, idx=None, obj_mask=None, evt_mask=None, fill: float = 0.0):
    """(value float32[N], local index int32[N]) of the n-th selected object of each event."""
    nev = len(offsets) - 1
    content = np.ascontiguousarray(content)
    out, oi = np.empty(nev, np.float32), np.empty(nev, np.int32)
    _check(lib().hepkref_get_in_offsets(offsets.ctypes.data, nev, content.ctypes.data, _dt(content), _p(obj_mask),
                                        _p(evt_mask), _p(idx), n, fill, out.ctypes.data, oi.ctypes.data))
    return out, oi


def set_in_offsets(offsets, content, value: float, n: int = 0, idx=None, obj_mask=None, evt_mask=None):
    """A copy of content (float32 or uint8) with the n-th selected object of each event set."""
    out = np.array(content, copy=True)
    dt = U8 if out.dtype == np.uint8 else _dt(out)
    _check(lib().hepkref_set_in_offsets(offsets.ctypes.data, len(offsets) - 1, out.ctypes.data, dt, _p(obj_mask),
                                        _p(evt_mask), _p(idx), n, value))
    return out


def select_opposite_sign(offsets, pt, charge, obj_mask=None) -> np.ndarray:
    pt = np.ascontiguousarray(pt)
    charge = np.ascontiguousarray(charge, np.int32)
    out = np.empty(int(offsets[-1]), np.uint8)
    _check(lib().hepkref_select_opposite_sign(offsets.ctypes.data, len(offsets) - 1, pt.ctypes.data, _dt(pt),
                                              charge.ctypes.data, _p(obj_mask), out.ctypes.data))
    return out


def compact(offsets, content, obj_mask=None) -> np.ndarray:
    content = np.ascontiguousarray(content)
    dt = U8 if content.dtype == np.uint8 else _dt(content)
    out = np.empty(max(1, int(offsets[-1])), content.dtype)
    n = C.c_int64()
    _check(lib().hepkref_compact(offsets.ctypes.data, len(offsets) - 1, content.ctypes.data, dt, _p(obj_mask),
                                 out.ctypes.data, C.byref(n)))
    return out[:n.value]


def p4(pt, eta, phi, mass):
    """(px, py, pz, E) float32 of each object (float64 arithmetic, rounded once)."""
    pt, eta, phi, mass = (np.ascontiguousarray(a) for a in (pt, eta, phi, mass))
    n = len(pt)
    o = [np.empty(n, np.float32) for _ in range(4)]
    _check(lib().hepkref_p4(pt.ctypes.data, eta.ctypes.data, phi.ctypes.data, mass.ctypes.data, _dt(pt), n,
                            *[a.ctypes.data for a in o]))
    return tuple(o)


def best_triplet(offsets, px, py, pz, en, obj_mask=None, target: float = 172.0):
    """(mass float32[N], local indices int32[N, 3]) of the triplet closest to target."""
    nev = len(offsets) - 1
    arrs = [np.ascontiguousarray(a, np.float32) for a in (px, py, pz, en)]
    m, idx = np.empty(nev, np.float32), np.empty(3 * nev, np.int32)
    _check(lib().hepkref_best_triplet(offsets.ctypes.data, nev, *[a.ctypes.data for a in arrs], _p(obj_mask),
                                      target, m.ctypes.data, idx.ctypes.data))
    return m, idx.reshape(nev, 3)


def _coll(c, names):
    if c is None:
        return Coll(None, None, None, None, None), []
    keep = [c.offsets] + [c.cols[k] for k in names if k in c.cols]
    extra = None
    for k in ("iso", "btag"):
        if k in c.cols:
            extra = c.cols[k].ctypes.data
    return Coll(c.offsets.ctypes.data, c.cols["pt"].ctypes.data, c.cols["eta"].ctypes.data,
                c.cols["phi"].ctypes.data, extra), keep


def query_struct(q, keep: list) -> QueryS:
    """A datagen.Query as the oracle's struct; arrays it points to go into keep."""
    def arr(a):
        if a is None:
            return None
        a = np.ascontiguousarray(a, np.float32)
        keep.append(a)
        return a.ctypes.data
    sc = np.ascontiguousarray(q.scales, np.float32)
    eds = [np.ascontiguousarray(e, np.float32) for e in q.edges()]
    keep += [sc] + eds
    qs = QueryS(q.mu_pt, q.mu_abseta, q.mu_iso, q.el_pt, q.el_abseta, q.jet_pt,
                q.jet_abseta, q.dr, q.btag, q.min_mu, q.min_jet, q.min_b,
                len(sc), sc.ctypes.data)
    for h in range(3):
        qs.edges[h] = eds[h].ctypes.data
        qs.nbins[h] = len(eds[h]) - 1
    if q.pu is not None:
        qs.pu_edges, qs.pu_contents, qs.pu_nbins = arr(q.pu[0]), arr(q.pu[1]), len(q.pu[0]) - 1
    if q.sf is not None:
        qs.sf_edges, qs.sf_contents, qs.sf_nbins = arr(q.sf[0]), arr(q.sf[1]), len(q.sf[0]) - 1
    if q.jes is not None:
        ee, pe, d = q.jes
        qs.jes_mode = 1
        qs.jes_eta_edges, qs.jes_pt_edges, qs.jes_delta = arr(ee), arr(pe), arr(d)
        qs.jes_n_eta, qs.jes_n_pt = len(ee) - 1, len(pe) - 1
    return qs


def pipeline(ds, queries, want_sumw2: bool = False) -> List[List[tuple]]:
    """Run the analysis pass on a datagen.Dataset for a list of datagen.Query.

    Returns hists[q][v] = [(sumw, counts)] * 3 for (HT, leading pt, nJet),
    or [(sumw, counts, sumw2)] * 3 with want_sumw2.
    """
    keep = []
    jets, k1 = _coll(ds.jets, ("pt", "eta", "phi", "btag"))
    mus, k2 = _coll(ds.muons, ("pt", "eta", "phi", "iso"))
    els, k3 = _coll(ds.electrons, ("pt", "eta", "phi"))
    keep += k1 + k2 + k3
    npu = getattr(ds, "npu", None)
    dss = DatasetS(ds.n_events, F16 if ds.content_dtype == "f16" else F32,
                   jets, mus, els, ds.weight.ctypes.data, _p(npu))
    qarr = (QueryS * max(1, len(queries)))()
    out, ptr_s, ptr_c, ptr_w2 = [], [], [], []
    for i, q in enumerate(queries):
        qarr[i] = query_struct(q, keep)
        per_q = []
        for v in range(q.n_scale):
            per_v = []
            for h in range(3):
                nb = len(q.edges()[h]) - 1
                s = np.zeros(nb + 2, np.float64)
                c = np.zeros(nb + 2, np.uint64)
                w2 = np.zeros(nb + 2, np.float64)
                ptr_s.append(s.ctypes.data)
                ptr_c.append(c.ctypes.data)
                ptr_w2.append(w2.ctypes.data)
                per_v.append((s, c, w2) if want_sumw2 else (s, c))
            per_q.append(per_v)
        out.append(per_q)
    ps = (C.c_void_p * max(1, len(ptr_s)))(*ptr_s)
    pc = (C.c_void_p * max(1, len(ptr_c)))(*ptr_c)
    pw = (C.c_void_p * max(1, len(ptr_w2)))(*ptr_w2)
    _check(lib().hepkref_pipeline(C.byref(dss), qarr, len(queries), C.cast(ps, C.c_void_p),
                                  C.cast(pw, C.c_void_p) if want_sumw2 else None, C.cast(pc, C.c_void_p)))
    del keep
    return out


def pipeline_events(ds, q) -> List[dict]:
    """Per-event values of the analysis pass for one query, composed from the
    primitives above as Sec. III's steering code would chain them (object
    selection -> Delta-R cleaning -> per-event reductions -> event selection;
    Listing 1 defines the H_T sum).  Independent of hepkref_pipeline, which
    composes the same primitives in C.

    Returns, per jet-energy scale v of the query, a dict of numpy arrays over
    the events: n_mu, n_jet, n_b (int32), ht, lead (float32; lead = -inf when
    no jet is selected), passed (uint8) and the event weight (float32).
    """
    j, m, el = ds.jets, ds.muons, ds.electrons
    n = ds.n_events
    mcuts = [(m.cols["pt"], GT, q.mu_pt), (m.cols["eta"], ABS_LT, q.mu_abseta)]
    if "iso" in m.cols:
        mcuts.append((m.cols["iso"], LT, q.mu_iso))
    msel = select(mcuts, m.n_objects)
    n_mu = reduce(COUNT, m.offsets, obj_mask=msel)
    _, _, clean = match_dr(j.offsets, j.cols["eta"], j.cols["phi"], m.offsets, m.cols["eta"],
                           m.cols["phi"], q.dr, mask_b=msel)
    if el is not None:
        esel = select([(el.cols["pt"], GT, q.el_pt), (el.cols["eta"], ABS_LT, q.el_abseta)], el.n_objects)
        _, _, clean = match_dr(j.offsets, j.cols["eta"], j.cols["phi"], el.offsets, el.cols["eta"],
                               el.cols["phi"], q.dr, mask_a=clean, mask_b=esel)
    # float16 content widens exactly; the scaled pt is one float32 product
    pt = np.ascontiguousarray(j.cols["pt"]).astype(np.float32)
    has_bt = "btag" in j.cols
    # event weight: w, times the pileup lookup, times the product of the
    # selected muons' scale factors (each product rounded to float32)
    wev = np.ascontiguousarray(ds.weight, np.float32).copy()
    if q.pu is not None and getattr(ds, "npu", None) is not None:
        wev = wev * get_bin_contents(ds.npu, *q.pu)
    if q.sf is not None:
        sf = get_bin_contents(m.cols["pt"], *q.sf)
        wev = wev * reduce(PROD, m.offsets, sf, obj_mask=msel)
    delta = jes_delta(j.cols["pt"], j.cols["eta"], *q.jes) if q.jes is not None else None
    out = []
    for s in np.asarray(q.scales, np.float32):
        ptv = pt * (np.float32(1.0) + s * delta) if delta is not None else pt * np.float32(s)
        jsel = select([(ptv, GT, q.jet_pt), (j.cols["eta"], ABS_LT, q.jet_abseta)], j.n_objects,
                      mask_in=clean)
        n_jet = reduce(COUNT, j.offsets, obj_mask=jsel)
        ht = reduce(SUM, j.offsets, ptv, obj_mask=jsel)
        lead = reduce(MAX, j.offsets, ptv, obj_mask=jsel)
        evc = [(n_mu, GE, q.min_mu), (n_jet, GE, q.min_jet)]
        if has_bt:
            bsel = select([(j.cols["btag"], GT, q.btag)], j.n_objects, mask_in=jsel)
            n_b = reduce(COUNT, j.offsets, obj_mask=bsel)
            evc.append((n_b, GE, q.min_b))
        else:
            n_b = np.zeros(n, np.int32)
        out.append({"n_mu": n_mu, "n_jet": n_jet, "n_b": n_b, "ht": ht, "lead": lead,
                    "passed": select(evc, n), "weight": wev})
    return out
